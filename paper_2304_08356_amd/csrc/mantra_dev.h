// Shared device/host structures of the sweep kernels (library internal).
#pragma once
#include <stdint.h>

namespace mantra {

typedef unsigned long long u64;
typedef unsigned int u32;

constexpr int kWave = 64;
#ifndef MANTRA_KE
#define MANTRA_KE 1
#endif
constexpr int kE = MANTRA_KE;        // edges per lane per batch
#ifndef MANTRA_SWEEP_WPS
#define MANTRA_SWEEP_WPS 4               // sweep waves per SIMD the register budget is cut for
#endif
constexpr int kC = kWave * kE;       // batch capacity (edges or arcs)
constexpr int kFwN = 2 * kC;         // LDS forwarding / tail table slots
constexpr int kFwBits = kFwN == 128 ? 7 : (kFwN == 256 ? 8 : (kFwN == 512 ? 9 : 10));
static_assert((1 << kFwBits) == kFwN, "table size must be a power of two");
constexpr int kStats = 20;           // launch statistics words (LaunchArgs::stats)
constexpr int kOrderBuckets = 160;   // log-scale cost buckets of the launch order (4 per octave)
constexpr int kArcChunkBits = 18;    // arcs per chunk of the shared arc pool: 2^18 (8 MiB)
constexpr int64_t kArcChunk = 1ll << kArcChunkBits;
constexpr int kXtLds = 256;          // chunk-table entries a sweep workgroup keeps in LDS
constexpr u32 kHInf = 0xFFFFu;       // "unreached" hop count
constexpr u64 kUMax = ~0ull;

enum { OPT_SH = 0, OPT_FM = 1, OPT_SFM = 2, OPT_PFM = 3 };
enum { STREAM_PAIR = 0, STREAM_BOOT = 1, STREAM_RADE = 2, STREAM_SRC = 3, STREAMS_PER_GRAPH = 4 };
enum { MODE_PAIRS = 0, MODE_DISTANCES = 1, MODE_TRK = 2, MODE_RTB = 3 };
// path draws of the TRK estimator: stream kStreamTrk + (the pair's stream)
constexpr u64 kStreamTrk = 1ull << 20;

// record flags (public ones mirror mantra.h)
enum : u32 {
    REC_OVERFLOW = 1u,
    REC_SELFCHECK = 2u,   // flow conservation at the origin failed (internal error)
    REC_HOPS_LIMIT = 4u,
    REC_ARCS_LIMIT = 8u,  // arc buffer too small: pair re-run with a larger one
    REC_WIDE = 16u,       // counts beyond 64 bits, taken exactly by the multiword path
};

// multiword counts of the exact path for pairs whose 64-bit counts saturate
constexpr int kWide = 4;  // limbs of 64 bits: counts below 2^256

// per-slab state of the multiword path (one pair at a time per slab)
struct WideSlabs {
    u64 *ST;          // [ns][nmax]          forward {tag | hops << 32}
    u64 *SS;          // [ns][nmax][kWide]   forward count
    u64 *RT;          // [ns][nmax]          reverse {tag | level << 32}
    u64 *RA;          // [ns][nmax][kWide]   reverse suffix sum
    u64 *NV;          // [ns][nmax][kWide]   N(v), zero between pairs
    int32_t *touched; // [ns][nmax]
    u32 *TL;          // [ns][gmax]          per edge of a tick: tail hops (or none)
    u64 *TC;          // [ns][gmax][kWide]   per edge of a tick: tail count; per arc of a tick: B(head)
    u64 *AR;          // [ns][cap][3 + kWide] arcs {head | t << 32, edge | tail << 32, tl | hl << 16, count}
    u32 *hdr;         // [ns][4]             pair serial
    int64_t nmax, cap, gmax;
};

struct DevGraph {
    const int32_t *U, *V, *T;           // [m] sorted by (graph, t, dst, src); local node ids
    const int64_t *out_off;             // [n_total+1] global node -> out-edge times
    const int32_t *out_t;               // [m] ascending per node
    const int64_t *in_off;
    const int32_t *in_t;
    const int64_t *seg_eoff;            // [G+1]
    const int32_t *seg_noff;            // [G+1]
    const int32_t *perm;                // [n_total] input node id -> internal id (hubs first)
    int32_t n_total;
    int32_t G;
    int64_t m;
};

// one request's slice of a launch
struct DevReq {
    int32_t opt, t0, t1, c;
    u64 seed;
    int32_t stream;      // STREAM_PAIR or STREAM_BOOT (RNG mode)
    int32_t graph;       // -1: pairs spread over all graphs (packed RNG mode), else graph id
    int64_t base;        // stream index of the slice's first pair (see per_graph)
    int64_t qoff;        // first launch-pair slot of this request
    int64_t count;       // pairs of this request in the launch
    int64_t per_graph;   // graph = -1: index i is pair i % per_graph of graph i / per_graph
    double *Bsum, *Wsum, *Rsum, *Esum; // accumulators (device), may be null
    u64 *rstat;          // per-request counters: overflow, reachable, hops limit, window edges, arcs; may be null
    int32_t mode;        // MODE_PAIRS (f = N/sigma), MODE_TRK (f = visits of one sampled optimal path),
                         // MODE_RTB (slot i is a source s, f = mean over targets z of N_z/sigma_sz), or
                         // MODE_DISTANCES: slot i is a source drawn from STREAM_SRC, swept
                         // to the window's end without a target; its distances go to hist
    int32_t hist_len;    // MODE_DISTANCES: bins of hist (the last one takes every larger distance)
    u64 *hist;           // [hist_len] sampled (source, node) pairs by distance; [hist_len]: largest distance
};

struct DevSlabs {
    u64 *F;           // [ns][nmax][2]  forward {tag | h<<32, S}, then reverse {rtag | lvl<<32, acc}
    u64 *N;           // [ns][nmax]     zero between pairs
    u64 *AG;          // [ns][gmax][2]  long ticks: each head run's decision, at the run's first edge
    int32_t *touched; // [ns][nmax]
    u64 *arcs;        // [ns][cap][4]   per slab: cap x {head | t<<32}, then cap x {k | u<<32, tail count, tl | hl<<16}
    u64 *xarcs;       // [nchunks][4 kArcChunk] the shared arc chunks (same layout), taken by pairs beyond cap
    u32 *xfree;       // [xwords] bit c set: chunk c is free
    u32 *xtab;        // [ns][xmax] chunk ids a slab's pair holds, in arc order
    int64_t xwords, xmax;
    u64 *XS;          // [ns][gmax][2]  long ticks: each edge's tail state
    u64 *T;           // [ns][nmax][2]  RTB sources: first arrival of each reached node (allocated for them)
    unsigned char *BM;// [ns][nmax bits, in 16-byte words] reached / alive set (graphs whose bitmap is not in LDS)
    u32 *hdr;         // [ns][4]        pair serial
    int64_t nmax, cap, gmax;
};

struct LaunchArgs {
    DevGraph g;
    DevSlabs sl;
    const DevReq *reqs;
    int32_t nreq;
    int32_t lds_bitmap;      // 1: reached bitmap of nmax bits in LDS; 0: in the slabs' BM (global memory)
    int32_t hub_nodes;       // forward state of nodes < hub_nodes lives in LDS
    int64_t npairs;              // launch slots (grid sizes); the pairs are slots qbase..np-1
    const int64_t *npairs_dev;   // np read from device memory (graph replays), or null: np = npairs
    int64_t qbase;               // first slot this launch takes
    const int32_t *pg, *ps, *pz; // explicit pairs (or null: RNG mode)
    const int32_t *pq;           // explicit launch slot -> original pair number (retries), or null
    void *rec;                   // mantra_pair_record[npairs] or null
    double *node_f;              // dense per-pair node output [npairs][n_total] or null
    double *edge_f;              // dense per-pair edge output [npairs][m] or null
    u32 *work;                   // work counter, zero at launch
    u64 *stats;                  // [kStats] window edges, arcs, overflow, reachable, hops-limit, retries, selfcheck, touched nodes,
                                 // touched edges, slab busy ticks, last end, ~first start, largest pair serial, (unused),
                                 // batches that loaded state, batches skipped, clock ticks in forward sweeps, clock ticks in
                                 // reverse sweeps and finalize
    int32_t *retry;              // [1 + npairs] pairs whose arcs did not fit
    int32_t *wide;               // [1 + npairs] pairs whose counts saturated, for the multiword path
                                 // (null: they are reported as saturated)
    int32_t wide_fm;             // 1: fm pairs too
};

struct ReduceArgs {
    const double *W;      // [n]
    const double *R;      // [n][c]
    const double *B;      // [n]
    int64_t n;
    int32_t c;
    double *part;         // [blocks][2 + c]: max W, sum B, max R_j
};

}  // namespace mantra
