// Sweep kernels of the temporal-betweenness hot path (gfx950).
//
// One wavefront owns one sampled pair (s, z) at a time and runs, in order:
//   1. the forward sweep over the pair's window of the time-sorted edge stream
//      (counts of optimal walks per vertex appearance, Definition 1 and the
//      estimator of Section 4.1), recording the arcs of the appearance DAG
//      that can lie on an optimal walk;
//   2. the reverse dependency sweep over those arcs (backtracking along the
//      temporal DAG, as in the exact algorithms the paper builds on), which
//      gives N(v) and N(e), the number of optimal walks through v and e;
//   3. the accumulation of f = N / sigma into the estimator sums of
//      Algorithm 1 (B, W and the c Rademacher-weighted sums) and the
//      temporal-edge sums (Appendix A).
// A persistent grid of single-wave workgroups pulls pairs from a work counter.
//
// Forward state per node (u = tail, v = head of an edge at time t), read only
// from appearances committed at earlier times (strict paths):
//   sh/sfm: h = fewest hops over the node's appearances so far, S = number of
//           fewest-hop walks over the appearances at that minimum;
//   fm    : h as above (for the record), S = number of walks reaching the node
//           at any earlier time (the origin counts once for s);
//   pfm   : h = fewest hops among prefix-foremost walks, S = their number,
//           set once, at the node's earliest arrival.
// Commits of all edges at time t happen after all reads at time t.
//
// Counts saturate at 2^64-1 in the forward sweep.  The reverse sweep only
// runs when sigma did not saturate; every product and partial sum it forms
// then counts distinct optimal walks and stays below sigma, so plain 64-bit
// arithmetic is exact there (the fm visit counts N(v), which may exceed
// sigma, are checked for wrap-around).

#include <hip/hip_runtime.h>
#include <stdint.h>
#include "mantra_dev.h"

namespace mantra {

// ---------------------------------------------------------------- helpers

// The kernels' one by-value argument sits at offset 0 of the kernel-argument
// segment (constant memory).  The sweep reads its fields there, where they
// are used, through a copy of the segment pointer that the compiler cannot
// see through, taken once per pair: each field is then loaded per pair
// (scalar loads) instead of all 84 dwords being kept live across the sweep
// loops, which spilled scalar registers into vector-register lanes inside
// the hot loops.
typedef const __attribute__((address_space(4))) LaunchArgs KArgs;
__device__ __forceinline__ KArgs &launch_args() {
    KArgs *p = (KArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return *p;
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ u64 ballot(bool p) { return (u64)__ballot(p ? 1 : 0); }
__device__ __forceinline__ int mbcnt(u64 m) {
    return (int)__builtin_amdgcn_mbcnt_hi((u32)(m >> 32), __builtin_amdgcn_mbcnt_lo((u32)m, 0u));
}
__device__ __forceinline__ int rl32(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ u64 rl64(u64 x, int l) {
    return ((u64)(u32)__builtin_amdgcn_readlane((int)(x >> 32), l) << 32) |
           (u64)(u32)__builtin_amdgcn_readlane((int)(u32)x, l);
}
// 64-bit value of lane src (per-lane source, through ds_bpermute)
__device__ __forceinline__ u64 shfl64(u64 x, int src) {
    const u32 lo = (u32)__shfl((int)(u32)x, src);
    const u32 hi = (u32)__shfl((int)(u32)(x >> 32), src);
    return ((u64)hi << 32) | lo;
}
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ u64 uni64(u64 x) { return rl64(x, __builtin_amdgcn_readfirstlane(lane_id())); }

__device__ __forceinline__ u64 sat_add(u64 a, u64 b) { u64 c = a + b; return c < a ? kUMax : c; }

__device__ __forceinline__ u64 ld_agent(const u64 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// SplitMix64 (Steele, Lea, Flood 2014): the k-th output of a generator
// started at state x is mix(x + k * golden).
__device__ __forceinline__ u64 sm_mix(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ u64 rng_word(u64 seed, u64 stream, u64 i, u64 j) {
    const u64 g = 0x9E3779B97F4A7C15ull;
    u64 key = sm_mix(seed + (stream + 1) * g);
    return sm_mix(key + (4 * i + j + 1) * g);
}

// first index in [a, b) with arr[idx] >= x (b if none); wave-cooperative
__device__ int64_t wave_lower_bound(const int32_t *arr, int64_t a, int64_t b, int32_t x) {
    const int l = lane_id();
    while (b - a > kWave) {
        int64_t step = (b - a + kWave - 1) / kWave;
        int64_t p = a + (int64_t)l * step;
        bool ok = p < b;
        bool pred = ok && arr[p] < x;
        int c = __popcll(ballot(pred));
        int nv = __popcll(ballot(ok));
        if (c == 0) return a;
        int64_t na = a + (int64_t)(c - 1) * step + 1;
        int64_t nb = (c < nv) ? a + (int64_t)c * step : b;
        a = na;
        b = nb < b ? nb : b;
    }
    int64_t p = a + l;
    bool pred = p < b && arr[p] < x;
    return a + __popcll(ballot(pred));
}
__device__ __forceinline__ int64_t wave_upper_bound(const int32_t *arr, int64_t a, int64_t b, int32_t x) {
    if (x == INT32_MAX) return b;
    return wave_lower_bound(arr, a, b, x + 1);
}

// ------------------------------------------------------------ LDS layout

constexpr int kHeadSlots = 128;  // hashed lane masks of a batch's run heads
struct FwdLds {           // forward: reductions of multi-edge runs, head table
    u32 rmin[kWave];      // per run (by run-start lane): min hop candidate
    u64 rlo[kWave];       // per run: count sum, low 32-bit halves
    u64 rhi[kWave];       //                      high 32-bit halves
    u64 hmask[kHeadSlots];  // lanes of the run heads whose node hashes to the slot
};
__device__ __forceinline__ u32 head_slot(int32_t node) { return ((u32)node * 2654435761u) >> 25; }  // 7 bits
struct RevLds {           // reverse: tail state by node, per batch
    u64 tb_key[kFwN];
    u64 tb_acc[kFwN];
    u32 tb_lvl[kFwN];     // bit 31: valid
};
union TabLds { FwdLds f; RevLds r; };


__device__ __forceinline__ u32 hslot(u32 node) { return (node * 2654435761u) >> (32 - kFwBits); }

// stamped open-addressing table (reverse): lookup, -1 if absent
__device__ __forceinline__ int tab_find(const u64 *keys, u32 stamp, u32 node) {
    u32 sl = hslot(node);
    for (int it = 0; it < kFwN; ++it) {
        u64 k = keys[sl];
        if ((u32)(k >> 32) != stamp) return -1;
        if ((u32)k == node) return (int)sl;
        sl = (sl + 1) & (kFwN - 1);
    }
    return -1;
}
// find or insert; *fresh = 1 if this call inserted the key
__device__ __forceinline__ int tab_insert(u64 *keys, u32 stamp, u32 node, int *fresh) {
    u32 sl = hslot(node);
    u64 want = ((u64)stamp << 32) | node;
    *fresh = 0;
    for (int it = 0; it < kFwN; ++it) {
        u64 k = keys[sl];
        if ((u32)(k >> 32) == stamp) {
            if ((u32)k == node) return (int)sl;
            sl = (sl + 1) & (kFwN - 1);
            continue;
        }
        u64 old = atomicCAS((unsigned long long *)&keys[sl], (unsigned long long)k, (unsigned long long)want);
        if (old == k) { *fresh = 1; return (int)sl; }
    }
    return -1;
}
__device__ __forceinline__ void lds_sat_add(u64 *p, u64 x) {
    u64 cur = *p;
    for (;;) {
        u64 nv = sat_add(cur, x);
        u64 old = atomicCAS((unsigned long long *)p, (unsigned long long)cur, (unsigned long long)nv);
        if (old == cur) return;
        cur = old;
    }
}
__device__ __forceinline__ void glb_sat_add(u64 *p, u64 x) {
    u64 cur = ld_agent(p);
    for (;;) {
        u64 nv = sat_add(cur, x);
        u64 old = atomicCAS((unsigned long long *)p, (unsigned long long)cur, (unsigned long long)nv);
        if (old == cur) return;
        cur = old;
    }
}

// ------------------------------------------------------------ per pair context

struct Pair {
    int32_t opt, t0, t1, c;
    int32_t g, s, z, ng, noff;
    int64_t q;             // launch slot
    int64_t qout;          // output row (pair number)
    int64_t elo, ehi;      // graph's edge range
    int64_t lo, hi;        // window
    u64 lam;
    const DevReq *req;
    u32 tag;               // forward state words of this pair carry it
    u32 rtag;              // reverse state words (the same memory) carry this one
    bool level;            // sh / sfm: hop levels matter
    bool single;           // distances: one source, every node its target (z = -1, no arcs)
    u64 trk_key;           // TRK: key of the pair's path-draw stream
    u64 trk_i;             // TRK: the pair's index in it
};

// A slab's buffers.  Only the slab's index is held; every address is
// computed from the launch arguments where it is used (scalar loads from the
// kernel-argument segment, see launch_args), so that the pointers are not
// kept live in scalar registers across the sweep loops, which spilled them.
struct Slab {
    int64_t id;
    u32 *xtl;  // LDS: the first kXtLds entries of the slab's chunk table
    // forward {tag | hops << 32, count} per node; the reverse's state shares the words
    __device__ __forceinline__ u64 *F() const { KArgs &a = launch_args(); return a.sl.F + id * a.sl.nmax * 2; }
    __device__ __forceinline__ u64 *R() const { return F(); }
    __device__ __forceinline__ u64 *N() const { KArgs &a = launch_args(); return a.sl.N + id * a.sl.nmax; }
    __device__ __forceinline__ int32_t *touched() const {
        KArgs &a = launch_args();
        return a.sl.touched + id * a.sl.nmax;
    }
    __device__ __forceinline__ u64 *AG() const { KArgs &a = launch_args(); return a.sl.AG + id * a.sl.gmax * 2; }
    __device__ __forceinline__ u64 *XS() const { KArgs &a = launch_args(); return a.sl.XS + id * a.sl.gmax * 2; }
    // RTB: [nmax][2] first arrival {time | hops << 32, count} of each reached node
    __device__ __forceinline__ u64 *T() const { KArgs &a = launch_args(); return a.sl.T + id * a.sl.nmax * 2; }
    // the chunks this slab holds, in arc order: arc cap + j is in chunk
    // xt(j / kArcChunk); entries below kXtLds in LDS (no global load on the
    // arc paths), the rest (pairs of more than 2^26 arcs) in global memory
    __device__ __forceinline__ u32 *xtg() const { KArgs &a = launch_args(); return a.sl.xtab + id * a.sl.xmax; }
    __device__ __forceinline__ u32 xt(int64_t j) const { return j < kXtLds ? xtl[j] : xtg()[j]; }
    __device__ __forceinline__ void xt_set(int64_t j, u32 c) const {
        if (j < kXtLds) xtl[j] = c;
        else xtg()[j] = c;
    }
};

// forward state of the highest-degree nodes (internal ids below K) in LDS:
// hops and count, valid where the reached set has the node (no pair tag)
struct Hub {
    u32 *h;
    u64 *s;
    int32_t K;
};

// Arc i of the pair: in the slab's own buffer of cap arcs ({head | time << 32}
// words, then {edge | tail << 32, tail count, tl | hl << 16} triples), else
// in the shared chunks it took (the same layout per chunk).  Arc records are
// written and read only through these.
__device__ __forceinline__ u64 *arc_m(const Slab &S, int64_t i) {
    KArgs &a = launch_args();
    const int64_t cap = a.sl.cap;
    if (i < cap) return a.sl.arcs + S.id * cap * 4 + i;
    const int64_t j = i - cap;
    return a.sl.xarcs + (int64_t)S.xt(j >> kArcChunkBits) * (4 * kArcChunk) + (j & (kArcChunk - 1));
}
// both words of arc i at once (one address computation)
struct ArcP { u64 *m, *x; };
__device__ __forceinline__ ArcP arc_at(const Slab &S, int64_t i) {
    KArgs &a = launch_args();
    const int64_t cap = a.sl.cap;
    ArcP r;
    if (i < cap) {
        r.m = a.sl.arcs + S.id * cap * 4 + i;
        r.x = a.sl.arcs + S.id * cap * 4 + cap + 3 * i;
    } else {
        const int64_t j = i - cap;
        u64 *c = a.sl.xarcs + (int64_t)S.xt(j >> kArcChunkBits) * (4 * kArcChunk);
        r.m = c + (j & (kArcChunk - 1));
        r.x = c + kArcChunk + 3 * (j & (kArcChunk - 1));
    }
    return r;
}
__device__ __forceinline__ u64 *arc_x(const Slab &S, int64_t i) {
    KArgs &a = launch_args();
    const int64_t cap = a.sl.cap;
    if (i < cap) return a.sl.arcs + S.id * cap * 4 + cap + 3 * i;
    const int64_t j = i - cap;
    return a.sl.xarcs + (int64_t)S.xt(j >> kArcChunkBits) * (4 * kArcChunk) + kArcChunk + 3 * (j & (kArcChunk - 1));
}

struct FwdOut {
    bool reached;
    u32 zh;
    u64 zS;
    int32_t t_arr;
    int64_t arcs;
    int64_t swept;
    u32 flags;
    int64_t reached_n;    // single source: nodes listed in the slab's touched list
    u32 live, dead;       // batches that loaded state, batches skipped (no reached tail)
    int64_t room;         // arcs the slab's buffer and its chunks hold
    int32_t nch;          // shared chunks the pair holds
};

__device__ __forceinline__ u32 ld_agent32(const u32 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Takes one free chunk of the launch's shared arc pool (a bitmap of free
// chunks, bit set = free): the wave scans the map from a per-slab offset, 64
// words at a time, and claims a set bit with an atomic AND.  Each word is
// tried until its bits run out, so the scan ends; -1 if no chunk is free.
__device__ int32_t chunk_take(KArgs &a, int32_t slab) {
    const int l = lane_id();
    const int64_t words = a.sl.xwords;
    if (words <= 0) return -1;
    const int64_t start = ((int64_t)slab * 97) % words;
    for (int64_t base = 0; base < words; base += kWave) {
        const bool valid = base + l < words;
        int64_t w = start + base + l;
        if (w >= words) w -= words;
        const u32 x = valid ? ld_agent32(&a.sl.xfree[w]) : 0u;
        u64 mk = ballot(x != 0u);
        while (mk) {
            const int src = __ffsll((long long)mk) - 1;
            mk &= mk - 1;
            u32 xw = (u32)rl32((int)x, src);
            const int64_t ww = base + src + start >= words ? base + src + start - words : base + src + start;
            while (xw) {
                const int b = __ffs((int)xw) - 1;
                u32 old = 0;
                if (l == 0)
                    old = __hip_atomic_fetch_and(&a.sl.xfree[ww], ~(1u << b), __ATOMIC_ACQUIRE,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                old = (u32)rl32((int)old, 0);
                if (old & (1u << b)) return (int32_t)(ww * 32 + b);
                xw = old & ~(1u << b);
            }
        }
    }
    return -1;
}

// Room for the pair's arcs [0, need): takes shared chunks while the slab's
// buffer and its chunks hold fewer.  false (the pair is then re-run with a
// buffer for every edge) if none is free.  Wave-uniform.
__device__ bool arc_room(KArgs &a, const Slab &S, FwdOut &o, int64_t need) {
    while (need > o.room) {
        if (o.nch >= a.sl.xmax) return false;
        const int32_t c = chunk_take(a, (int32_t)S.id);
        if (c < 0) return false;
        if (lane_id() == 0) S.xt_set(o.nch, (u32)c);
        o.nch += 1;
        o.room += kArcChunk;
        __syncthreads();  // every lane's arc addresses read the new table entry
    }
    return true;
}

// gives the pair's chunks back (after every read of its arcs)
__device__ void chunks_free(KArgs &a, const Slab &S, int32_t nch) {
    if (nch <= 0) return;
    __threadfence();
    for (int i = lane_id(); i < nch; i += kWave) {
        const u32 c = S.xt(i);
        __hip_atomic_fetch_or(&a.sl.xfree[c >> 5], 1u << (c & 31), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The pair's reached set (forward), then its alive set (reverse): a bitmap
// of the nodes, bit v of word v / 32.  On graphs of up to 65,536 nodes it is
// in LDS.  Larger graphs keep it in the slab's global memory (GBM), set with
// atomic ORs (performed in L2) and read with loads that bypass L1 (so a
// line L1 holds can never hide a bit the wave set); a wave's memory
// operations are performed in order, so it sees its own bits.  At 2*10^6
// nodes the map is 256 KB per slab, and the words of the nodes most windows
// touch stay in L2.  Cleared at the start of each pair and before each
// reverse sweep.
template <bool GBM>
__device__ __forceinline__ u32 bm_word(const u32 *bm, int32_t v) {
    if (GBM) return ld_agent32(&bm[v >> 5]);
    return bm[v >> 5];
}
template <bool GBM>
__device__ __forceinline__ bool rch_test(const u32 *bm, int32_t v) {
    return (bm_word<GBM>(bm, v) >> (v & 31)) & 1u;
}
template <bool GBM>
__device__ __forceinline__ void rch_set(u32 *bm, int32_t v) {
    if (GBM) __hip_atomic_fetch_or(&bm[v >> 5], 1u << (v & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else atomicOr(&bm[v >> 5], 1u << (v & 31));
}

// (room for pos was made by arc_room)
__device__ __forceinline__ void put_arc(const Slab &S, int64_t pos, int32_t v, int32_t t, u32 k,
                                        int32_t u, u64 tc, u32 tl, u32 hl) {
    *arc_m(S, pos) = (u64)(u32)v | ((u64)(u32)t << 32);
    u64 *x = arc_x(S, pos);
    x[0] = (u64)k | ((u64)(u32)u << 32);
    x[1] = tc;
    x[2] = (u64)tl | ((u64)hl << 16);
}

// decide the commit of head v at time t given its run's (d, c) and its
// current state (reached, hv, Sv); returns useful, sets the new state
__device__ __forceinline__ bool head_commit(int opt, bool rv, u32 hv, u64 Sv, u32 d, u64 c,
                                            int32_t v, int32_t z, u32 zh, u32 *nh, u64 *nS) {
    if (opt == OPT_SH || opt == OPT_SFM) {
        u32 hcur = rv ? hv : kHInf;
        bool useful = d <= hcur;
        if (opt == OPT_SH && zh != kHInf) {
            if (v != z && d >= zh) useful = false;
            if (v == z && d > zh) useful = false;
        }
        if (!useful) return false;
        if (d < hcur) { *nh = d; *nS = c; }
        else { *nh = hcur; *nS = sat_add(Sv, c); }
        return true;
    }
    if (opt == OPT_FM) {
        u32 hcur = rv ? hv : kHInf;
        *nh = d < hcur ? d : hcur;
        *nS = sat_add(rv ? Sv : 0, c);
        return true;
    }
    // pfm: only the earliest arrival counts
    if (rv) return false;
    *nh = d;
    *nS = c;
    return true;
}

// ------------------------------------------------------------ forward: long tick
// A tick of more edges than one row of 64 forms a batch of its own.  Every
// edge of a tick reads the state from before the tick, so the reads of all
// its rows can go out at once, and the tick's commits follow once every read
// is done.  The tick's edges are sorted by head, so the edges of one head
// form one contiguous run; a run's candidate (min hops, count) is reduced by a
// segmented scan across the lanes, row after row, with the partial of a run
// that continues into the next row carried in wave-uniform registers.  Ticks
// of up to two rows are held in registers (fwd_tick2); longer ones keep the
// per-edge tail state and the per-run decisions in the slab's scratch XS / AG
// between a read pass and a commit pass (fwd_long_tick).

// forward modes: a pair (arcs, stop at z); a source's distances (no arcs,
// first-arrival hops in N); a source for the RTB estimator (arcs, and each
// node's first arrival {time | hops << 32, count} in T)
enum { FWD_PAIR = 0, FWD_DIST = 1, FWD_RTB = 2 };

__device__ __forceinline__ u64 shfl_up64(u64 x, int off) {
    const u32 lo = (u32)__shfl_up((int)(u32)x, off);
    const u32 hi = (u32)__shfl_up((int)(u32)(x >> 32), off);
    return ((u64)hi << 32) | lo;
}

// (d, c) <- (d, c) + (d2, c2) over one head's candidates: the fewest hops d and
// the count of the walks that reach the head with them (sh / sfm), or the
// fewest hops and the count over every reached tail (fm / pfm)
__device__ __forceinline__ void cand_join(bool level, u32 &d, u64 &c, u32 d2, u64 c2) {
    if (!level) { d = d2 < d ? d2 : d; c = sat_add(c, c2); return; }
    if (d2 < d) { d = d2; c = c2; }
    else if (d2 == d) c = sat_add(c, c2);
}

// Segmented inclusive scan of (d, c) over the lanes of one row: st = lane of
// my run's start in the row (-1: the run started in an earlier row, whose
// partial (cd, cc) is joined).  A run-end lane then holds its run's total.
__device__ __forceinline__ void run_scan(bool level, bool multi, int st, u32 cd, u64 cc, u32 &d, u64 &c) {
    const int l = lane_id();
    if (multi) {
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const u32 d2 = (u32)__shfl_up((int)d, off);
            const u64 c2 = shfl_up64(c, off);
            if (l - off >= st && l >= off) cand_join(level, d, c, d2, c2);
        }
    }
    if (st < 0) cand_join(level, d, c, cd, cc);
}

// the tail state (hops, count) of a lane from its loaded words (hops kHInf:
// not reached); the hub's LDS copy for hub nodes
__device__ __forceinline__ void state_of(const Pair &P, const Hub &H, bool maybe, int32_t x, u64 th, u64 ts,
                                         u32 lh, u64 ls, u32 &h, u64 &c) {
    const bool hub = x < H.K;
    h = !maybe ? kHInf : hub ? lh : ((u32)th == P.tag) ? ((u32)(th >> 32) & 0xFFFFu) : kHInf;
    c = hub ? ls : ts;
}

// a committed head: its new state and the reached set
template <bool GBM>
__device__ __forceinline__ void head_store(const Pair &P, const Slab &S, u32 *bm, const Hub &H, int32_t v,
                                           u32 nh, u64 nS) {
    if (v < H.K) { H.h[v] = nh; H.s[v] = nS; }
    else {
        u64 *const Fp = S.F();
        Fp[2 * (int64_t)v] = (u64)P.tag | ((u64)nh << 32);
        Fp[2 * (int64_t)v + 1] = nS;
    }
    rch_set<GBM>(bm, v);
}
// single source: the first arrivals of a row (the list of reached nodes, and
// the hops (distances) or the first arrival (RTB) committed there)
template <int FM>
__device__ __forceinline__ void first_arrivals(const Pair &P, const Slab &S, FwdOut &o, bool fa, int32_t v,
                                               int32_t t, u32 nh, u64 nS) {
    if (FM == FWD_PAIR) return;
    const u64 fm_ = ballot(fa);
    if (fa) {
        if (FM == FWD_DIST && P.opt != OPT_SH) S.N()[v] = (u64)nh + 1ull;
        if (FM == FWD_RTB) {
            u64 *const Tp = S.T();
            Tp[2 * (int64_t)v] = (u64)(u32)t | ((u64)nh << 32);
            Tp[2 * (int64_t)v + 1] = nS;
        }
        S.touched()[o.reached_n + mbcnt(fm_)] = v;
    }
    o.reached_n += __popcll(fm_);
}

// a tick of 65..128 edges at g0 (ur / vr: tail and head of edge g0 + 64 r +
// lane; head -1 past g1)
template <int FM, bool GBM>
__device__ void fwd_tick2(KArgs &a, const Pair &P, const Slab &S, u32 *bm, const Hub &H,
                          int64_t g0, int64_t g1, int32_t t, const int32_t (&ur)[2], const int32_t (&vr)[2],
                          FwdOut &o, u32 &zh, u64 &zS, bool &zhit) {
    constexpr int R = 2;
    u64 *const Fp = S.F();
    const int l = lane_id();
    const int opt = P.opt;
    const u64 le = (l == kWave - 1) ? kUMax : ((2ull << l) - 1ull);  // lanes <= l
    const u64 ge = ~((1ull << l) - 1ull);                             // lanes >= l
    const u32 kBig = 0xFFFFFFFFu;
    bool rs[R], re[R], rt[R], hr[R];
    u64 any = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool act = g0 + r * kWave + l < g1;
        int32_t vp = __shfl_up(vr[r], 1);
        int32_t vn = __shfl_down(vr[r], 1);
        if (l == 0) vp = r == 0 ? -2 : rl32(vr[r - 1 < 0 ? 0 : r - 1], kWave - 1);
        if (l == kWave - 1) vn = r + 1 < R ? rl32(vr[r + 1 < R ? r + 1 : r], 0) : -1;
        rs[r] = act && vr[r] != vp;
        re[r] = act && vr[r] != vn;
        if (GBM) {
            // reached set in global memory: no bitmap loads here; every lane
            // loads its nodes' state words, whose pair tag (or, for hubs,
            // hops kHInf: cleared at the pair's start) decides whether the
            // node was reached
            rt[r] = act;
            hr[r] = re[r];
        } else {
            const bool dead = opt == OPT_PFM && act && rch_test<GBM>(bm, vr[r]);
            rt[r] = act && !dead && rch_test<GBM>(bm, ur[r]);
            hr[r] = re[r] && !dead && rch_test<GBM>(bm, vr[r]);
            any |= ballot(rt[r]);
        }
    }
    if (!GBM && !any) { o.dead += 1; return; }
    // the state before the tick: every lane loads (see the batch path), both
    // rows at once, then each word is decoded
    u64 thu[R], tsu[R], thv[R], tsv[R];
    u32 lhu[R], lhv[R];
    u64 lsu[R], lsv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t iu = (rt[r] && ur[r] >= H.K) ? (int64_t)ur[r] : (int64_t)P.s;
        const int64_t iv = (hr[r] && vr[r] >= H.K) ? (int64_t)vr[r] : (int64_t)P.s;
        thu[r] = Fp[2 * iu];
        tsu[r] = Fp[2 * iu + 1];
        thv[r] = Fp[2 * iv];
        tsv[r] = Fp[2 * iv + 1];
        lhu[r] = 0; lhv[r] = 0; lsu[r] = 0; lsv[r] = 0;
        if (H.K > 0) {
            const int ju = ur[r] < H.K ? ur[r] : 0, jv = (vr[r] >= 0 && vr[r] < H.K) ? vr[r] : 0;
            lhu[r] = H.h[ju]; lsu[r] = H.s[ju];
            lhv[r] = H.h[jv]; lsv[r] = H.s[jv];
        }
    }
    u32 hu[R], hv[R];
    u64 su[R], sv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        state_of(P, H, rt[r], ur[r], thu[r], tsu[r], lhu[r], lsu[r], hu[r], su[r]);
        state_of(P, H, hr[r], vr[r], thv[r], tsv[r], lhv[r], lsv[r], hv[r], sv[r]);
    }
    if (ballot((hu[0] != kHInf && hu[0] + 1 >= kHInf) || (hu[1] != kHInf && hu[1] + 1 >= kHInf))) {
        o.flags |= REC_HOPS_LIMIT;
        return;
    }
    if (GBM && !ballot(hu[0] != kHInf || hu[1] != kHInf)) { o.dead += 1; return; }
    o.live += 1;
    // per run: the candidate over its tails, then its head's decision; every
    // read of the tick is done, so a run's commit follows at once
    u32 mine[R];   // at run ends: d | commit << 31
    u32 cd = kBig;
    u64 cc = 0;
    u32 zh_new = zh;
    u64 zS_new = zS;
    bool zany = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        u32 d = hu[r] != kHInf ? hu[r] + 1 : kBig;
        u64 c = hu[r] != kHInf ? su[r] : 0ull;
        const u64 below = ballot(rs[r]) & le;
        const int st = below ? 63 - __clzll((long long)below) : -1;
        const bool multi = ballot((g0 + r * kWave + l < g1) && !(rs[r] && re[r])) != 0;
        run_scan(P.level, multi, st, cd, cc, d, c);
        // the row's last run continues into the next row
        if (g0 + r * kWave + kWave - 1 < g1 && !(ballot(re[r]) >> (kWave - 1))) {
            cd = (u32)rl32((int)d, kWave - 1);
            cc = rl64(c, kWave - 1);
        } else { cd = kBig; cc = 0; }
        u32 nh = 0;
        u64 nS = 0;
        const bool ok = re[r] && d != kBig &&
                        head_commit(opt, hv[r] != kHInf, hv[r], sv[r], d, c, vr[r], P.z, zh, &nh, &nS);
        if (ok) head_store<GBM>(P, S, bm, H, vr[r], nh, nS);
        first_arrivals<FM>(P, S, o, ok && hv[r] == kHInf, vr[r], t, nh, nS);
        const u64 zm = ballot(ok && vr[r] == P.z);
        if (zm) {
            const int zl = __ffsll((long long)zm) - 1;
            zh_new = (u32)rl32((int)nh, zl);
            zS_new = rl64(nS, zl);
            zany = true;
        }
        mine[r] = ok ? (d | 0x80000000u) : 0u;
    }
    // each edge learns its run's decision (d, commit) from the run's end
    // lane, in its row or, for a run that continues, in the next one
    u32 okd[R];
    u32 back = 0;
#pragma unroll
    for (int r = R - 1; r >= 0; --r) {
        const u64 m = ballot(re[r]) & ge;
        const int src = m ? __ffsll((long long)m) - 1 : l;
        u32 x = (u32)__shfl((int)mine[r], src);
        if (!m) x = back;
        okd[r] = x;
        back = (u32)rl32((int)x, 0);
    }
    // arcs in edge order
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const u32 dd = okd[r] & 0x7FFFFFFFu;
        const bool rec = FM != FWD_DIST && hu[r] != kHInf && (okd[r] >> 31) && (!P.level || hu[r] + 1 == dd);
        const u64 m = ballot(rec);
        if (m) {
            if (!arc_room(a, S, o, o.arcs + __popcll(m))) { o.flags |= REC_ARCS_LIMIT; return; }
            if (rec) put_arc(S, o.arcs + mbcnt(m), vr[r], t, (u32)(g0 + r * kWave + l), ur[r], su[r], hu[r], dd);
            o.arcs += __popcll(m);
        }
    }
    if (zany) {
        if (opt == OPT_SH) { if (zh_new < zh) o.t_arr = t; }
        else o.t_arr = t;
        zh = zh_new;
        zS = zS_new;
        zhit = true;
    }
}

// a tick of more than 128 edges [g0, g1): a read pass that keeps each edge's
// tail state {hops | reached << 32 | run start << 33, count} in XS and each
// run's decision {d | new hops << 32 | first arrival << 62 | commit << 63,
// new count} in AG at the run's first edge, then a commit pass
template <int FM, bool GBM>
__device__ void fwd_long_tick(KArgs &a, const Pair &P, const Slab &S, u32 *bm, const Hub &H,
                              int64_t g0, int64_t g1, int32_t t, FwdOut &o, u32 &zh, u64 &zS, bool &zhit) {
    u64 *const Fp = S.F();
    u64 *const XSp = S.XS();
    u64 *const AGp = S.AG();
    const int l = lane_id();
    const int opt = P.opt;
    const int32_t *U = a.g.U, *V = a.g.V;
    const u64 le = (l == kWave - 1) ? kUMax : ((2ull << l) - 1ull);  // lanes <= l
    const u32 kBig = 0xFFFFFFFFu;
    u32 cd = kBig;       // partial of the run that continues into the row
    u64 cc = 0;
    int64_t cs = g0;     // its first edge
    int32_t cv = -2;     // head of the previous row's last edge
    bool any = false;
    for (int64_t sb = g0; sb < g1; sb += kWave) {
        const int64_t idx = sb + l;
        const bool act = idx < g1;
        const int32_t u = act ? U[idx] : 0, v = act ? V[idx] : -1;
        const int32_t vnx = sb + kWave < g1 ? V[sb + kWave] : -1;
        int32_t vp = __shfl_up(v, 1);
        int32_t vn = __shfl_down(v, 1);
        if (l == 0) vp = cv;
        if (l == kWave - 1) vn = vnx;
        const bool rs = act && v != vp, re = act && v != vn;
        const bool dead = opt == OPT_PFM && act && rch_test<GBM>(bm, v);
        const bool rt = act && !dead && rch_test<GBM>(bm, u);
        const bool hr = re && !dead && rch_test<GBM>(bm, v);
        const int64_t iu = (rt && u >= H.K) ? (int64_t)u : (int64_t)P.s;
        const int64_t iv = (hr && v >= H.K) ? (int64_t)v : (int64_t)P.s;
        const u64 thu = Fp[2 * iu], tsu = Fp[2 * iu + 1], thv = Fp[2 * iv], tsv = Fp[2 * iv + 1];
        u32 lhu = 0, lhv = 0;
        u64 lsu = 0, lsv = 0;
        if (H.K > 0) {
            const int ju = u < H.K ? u : 0, jv = (v >= 0 && v < H.K) ? v : 0;
            lhu = H.h[ju]; lsu = H.s[ju];
            lhv = H.h[jv]; lsv = H.s[jv];
        }
        u32 hu, hv;
        u64 su, sv;
        state_of(P, H, rt, u, thu, tsu, lhu, lsu, hu, su);
        if (ballot(hu != kHInf && hu + 1 >= kHInf)) { o.flags |= REC_HOPS_LIMIT; return; }
        u32 d = hu != kHInf ? hu + 1 : kBig;
        u64 c = hu != kHInf ? su : 0ull;
        const u64 below = ballot(rs) & le;
        const int st = below ? 63 - __clzll((long long)below) : -1;
        run_scan(P.level, ballot(act && !(rs && re)) != 0, st, cd, cc, d, c);
        state_of(P, H, hr, v, thv, tsv, lhv, lsv, hv, sv);
        u32 nh = 0;
        u64 nS = 0;
        const bool ok = re && d != kBig && head_commit(opt, hv != kHInf, hv, sv, d, c, v, P.z, zh, &nh, &nS);
        const int64_t k = (st >= 0 ? sb + st : cs) - g0;
        if (re)
            AGp[2 * k] = (u64)d | ((u64)nh << 32) | ((u64)(ok && hv == kHInf) << 62) | ((u64)ok << 63);
        if (re) AGp[2 * k + 1] = nS;
        if (act) {
            XSp[2 * (idx - g0)] = (u64)hu | ((u64)(hu != kHInf) << 32) | ((u64)rs << 33);
            XSp[2 * (idx - g0) + 1] = su;
        }
        any = any || ballot(ok) != 0;
        const int st63 = rl32(st, kWave - 1);
        if (ballot(l == kWave - 1 && act && !re)) {
            cd = (u32)rl32((int)d, kWave - 1);
            cc = rl64(c, kWave - 1);
            if (st63 >= 0) cs = sb + st63;
        } else { cd = kBig; cc = 0; }
        cv = rl32(v, kWave - 1);
    }
    if (!any) { o.dead += 1; return; }
    o.live += 1;
    __syncthreads();
    u32 zh_new = zh;
    u64 zS_new = zS;
    bool zany = false;
    u64 cr0 = 0, cr1 = 0;  // decision of the run that continues into the row
    for (int64_t sb = g0; sb < g1; sb += kWave) {
        const int64_t idx = sb + l;
        const bool act = idx < g1;
        const int64_t i = act ? idx - g0 : 0;
        const u64 x0 = act ? XSp[2 * i] : 0ull, su = act ? XSp[2 * i + 1] : 0ull;
        const u64 a0 = act ? AGp[2 * i] : 0ull, a1 = act ? AGp[2 * i + 1] : 0ull;
        const int32_t u = act ? U[idx] : 0, v = act ? V[idx] : 0;
        const bool rs = act && ((x0 >> 33) & 1ull);
        const u64 below = ballot(rs) & le;
        const int st = below ? 63 - __clzll((long long)below) : 0;
        u64 r0 = shfl64(a0, st), r1 = shfl64(a1, st);
        if (!below) { r0 = cr0; r1 = cr1; }
        const bool okr = act && (r0 >> 63);
        const u32 dd = (u32)r0;
        const u32 nh = (u32)(r0 >> 32) & 0xFFFFu;
        const bool ok = rs && okr;
        if (ok) head_store<GBM>(P, S, bm, H, v, nh, r1);
        first_arrivals<FM>(P, S, o, ok && ((r0 >> 62) & 1ull), v, t, nh, r1);
        const u64 zm = ballot(ok && v == P.z);
        if (zm) {
            const int zl = __ffsll((long long)zm) - 1;
            zh_new = (u32)rl32((int)nh, zl);
            zS_new = rl64(r1, zl);
            zany = true;
        }
        const u32 hu = (u32)x0;
        const bool rec = FM != FWD_DIST && okr && ((x0 >> 32) & 1ull) && (!P.level || hu + 1 == dd);
        const u64 m = ballot(rec);
        if (m) {
            if (!arc_room(a, S, o, o.arcs + __popcll(m))) { o.flags |= REC_ARCS_LIMIT; return; }
            if (rec) put_arc(S, o.arcs + mbcnt(m), v, t, (u32)idx, u, su, hu, dd);
            o.arcs += __popcll(m);
        }
        cr0 = rl64(r0, kWave - 1);
        cr1 = rl64(r1, kWave - 1);
    }
    if (zany) {
        if (opt == OPT_SH) { if (zh_new < zh) o.t_arr = t; }
        else o.t_arr = t;
        zh = zh_new;
        zS = zS_new;
        zhit = true;
    }
    __syncthreads();
}

// ------------------------------------------------------------ forward sweep

// edges of the batch at b: lane l holds edge b + l (past the window: time
// INT32_MAX, head -1); tnext = time of edge b + 64, INT32_MAX past the window
__device__ __forceinline__ void load_batch(KArgs &a, const Pair &P, int64_t b, int32_t &t, int32_t &u,
                                           int32_t &v, int32_t &tnext) {
    const int l = lane_id();
    const int64_t i = b + l;
    const bool ld = i < P.hi;
    t = ld ? a.g.T[i] : INT32_MAX;
    u = ld ? a.g.U[i] : 0;
    v = ld ? a.g.V[i] : -1;
    tnext = (b + kWave < P.hi) ? a.g.T[b + kWave] : INT32_MAX;
}

// Forward sweep of one pair over its window [P.lo, P.hi), in batches of up to
// 64 edges (one per lane) that hold whole ticks; a tick longer than 64 edges
// is a batch of its own (fwd_tick2, fwd_long_tick).  Within a batch, the edges of tick
// tau read the state committed before tau: the state at batch start (loaded
// from the slab) or the commit of an earlier tick of the same batch, passed
// from the committing lane's registers.  Maximal runs of ticks that read no
// commit made inside the run ("segments") are processed together.
template <int FM, bool GBM>
__device__ void forward(KArgs &a, const Pair &P, const Slab &S, u32 *bm, const Hub &H, FwdLds &L,
                        FwdOut &o) {
    u64 *const Fp = S.F();
    u64 *const Np = S.N();
    u64 *const Tp = S.T();
    int32_t *const Tch = S.touched();
    constexpr bool SINGLE = FM != FWD_PAIR;
    static_assert(kE == 1, "the forward sweep is written for one edge per lane");
    const int l = lane_id();
    const int opt = P.opt;
    const u64 le = (l == kWave - 1) ? kUMax : ((2ull << l) - 1ull);  // lanes <= l
    const u32 kBig = 0xFFFFFFFFu;
    u32 zh = kHInf;
    u64 zS = 0;
    bool zhit = false;
    bool done = false;
    int64_t b0 = P.lo;
    o.arcs = 0;
    o.flags = 0;
    o.t_arr = -1;
    int32_t t, u, v, tnext;
    load_batch(a, P, b0, t, u, v, tnext);
    // Reached set in global memory (GBM): the bitmap words of a batch's tails
    // and heads are loaded during the batch before it, ahead of that batch's
    // commits (pref), and the nodes those commits reached first are patched
    // in from registers (pu, pv): the reached test of a batch then waits for
    // no load.  (One wave's memory operations are performed in order, so bits
    // set by earlier batches are seen.)
    u32 bu = 0, bv = 0;
    bool pref = false, pu = false, pv = false;
    while (b0 < P.hi && !done) {
        // ---- batch: up to 64 edges, whole ticks
        const int64_t avail = P.hi - b0;
        const int nb = avail < kWave ? (int)avail : kWave;
        int nbat = nb;
        if (nb == kWave && b0 + kWave < P.hi) {
            const int32_t tlast = rl32(t, kWave - 1);
            if (tnext == tlast) {
                const int first = __ffsll((long long)ballot(t == tlast)) - 1;
                if (first == 0) {
                    // one tick longer than a batch: its second row, and its end
                    const int64_t i1 = b0 + kWave + l;
                    const bool in1 = i1 < P.hi;
                    const int32_t t1 = in1 ? a.g.T[i1] : INT32_MAX;
                    int32_t ur[2] = {u, in1 ? a.g.U[i1] : 0};
                    int32_t vr[2] = {v, in1 ? a.g.V[i1] : -1};
                    const u64 mt = ballot(t1 == tlast);
                    int64_t g1;
                    if (~mt) {
                        g1 = b0 + kWave + (__ffsll((long long)~mt) - 1);
                        if (t1 != tlast) { ur[1] = 0; vr[1] = -1; }
                    } else {
                        // no tick is longer than the graph's longest one
                        const int64_t lim = b0 + a.sl.gmax + 1 < P.hi ? b0 + a.sl.gmax + 1 : P.hi;
                        g1 = wave_upper_bound(a.g.T, b0 + 2 * kWave, lim, tlast);
                    }
                    __syncthreads();
                    pref = false;  // the batch after the tick loads its own words
                    if (g1 - b0 <= 2 * kWave) fwd_tick2<FM, GBM>(a, P, S, bm, H, b0, g1, tlast, ur, vr, o, zh, zS, zhit);
                    else fwd_long_tick<FM, GBM>(a, P, S, bm, H, b0, g1, tlast, o, zh, zS, zhit);
                    o.swept = g1 - P.lo;
                    b0 = g1;
                    if (o.flags & (REC_HOPS_LIMIT | REC_ARCS_LIMIT)) return;
                    if (zhit && opt != OPT_SH) done = true;
                    __syncthreads();
                    load_batch(a, P, b0, t, u, v, tnext);
                    continue;
                }
                nbat = first;
            }
        }
        const bool in = l < nbat;
        int32_t tp = __shfl_up(t, 1);
        int32_t vp = __shfl_up(v, 1);
        if (l == 0) { tp = INT32_MIN; vp = -2; }
        const bool gst = in && t != tp;
        const bool rs = in && (gst || v != vp);
        const u64 gm = ballot(gst);
        const u64 rsall = ballot(rs);
        const int tid = __popcll(gm & le) - 1;
        const int ntick = __popcll(gm);
        const int rsl = 63 - __clzll((long long)((rsall & le) | 1ull));  // lane of my run's start
        // ---- state at batch start.  A set bit of the reached set is exactly
        // a node whose state this pair wrote: the reached test needs no load
        // of the state, and the state loads of a live batch are in flight
        // while its dependencies are worked out.
        // (thu, su) / (thv, sv): the slab's {tag | hops << 32, count} words;
        // the hops are taken out where they are first used, so that nothing
        // waits for the loads before then.
        // pfm: a node's state is final at its first arrival, so an edge
        // whose head was reached before the batch can neither commit nor lie
        // on an optimal walk (its whole run is dead); its tail needs no load.
        bool ru, rv, tagm = false;
        if (GBM) {
            if (pref) {
                ru = ((bu >> (u & 31)) & 1u) || pu;
                rv = ((bv >> (v & 31)) & 1u) || pv;
            } else {
                // no words loaded ahead (a pair's first batch, or the batch
                // after a long tick): every lane loads its nodes' state words,
                // whose pair tag (hub nodes: hops kHInf) tells whether the
                // node was reached -- one round trip instead of two
                tagm = true;
                ru = in;
                rv = in;
            }
        } else {
            ru = in && rch_test<GBM>(bm, u);
            rv = in && rch_test<GBM>(bm, v);
        }
        pref = false;
        const bool dead = opt == OPT_PFM && in && rv && !tagm;
        const bool rt = in && !dead && ru;
        const bool hr = rs && rv;
        u64 thu = 0, thv = 0, su = 0, sv = 0;
        u32 lhu = 0, lhv = 0;
        u64 lsu = 0, lsv = 0;
        // the next batch's edges, in flight while this one is processed
        int32_t t2, u2, v2, tn2;
        load_batch(a, P, b0 + nbat, t2, u2, v2, tn2);
        // no tail reached at batch start: no tick of the batch can commit
        if (!ballot(rt)) {
            if (GBM) {
                // nothing is committed: the next batch's words need no patch
                bu = v2 >= 0 ? bm_word<GBM>(bm, u2) : 0u;
                bv = v2 >= 0 ? bm_word<GBM>(bm, v2) : 0u;
                pu = false; pv = false;
                pref = true;
            }
            b0 += nbat;
            o.swept = b0 - P.lo;
            t = t2; u = u2; v = v2; tnext = tn2;
            o.dead += 1;
            continue;
        }
        o.live += 1;
        {
            // every lane loads (lanes with nothing to load read the origin's
            // state, one line for all of them): no merge of a loaded value
            // with a default, so no early wait for the loads
            // hub nodes' state is in LDS (loaded for every lane, index 0 for
            // the others)
            const int64_t iu = (rt && u >= H.K) ? (int64_t)u : (int64_t)P.s;
            const int64_t iv = (hr && v >= H.K) ? (int64_t)v : (int64_t)P.s;
            thu = Fp[2 * iu];
            su = Fp[2 * iu + 1];
            thv = Fp[2 * iv];
            sv = Fp[2 * iv + 1];
            if (H.K > 0) {
                const int ju = u < H.K ? u : 0, jv = v < H.K ? v : 0;
                lhu = H.h[ju]; lsu = H.s[ju];
                lhv = H.h[jv]; lsv = H.s[jv];
            }
        }
        // ---- in-batch dependencies.  pred (hpred) = the latest run-head lane of
        // an earlier tick whose head is my tail (my head), or -1.  Every run
        // head publishes its node's state after its tick (committed or not),
        // so a lane reads its node's state from that one lane.  The lanes come
        // from a table of head-lane masks hashed by node (LDS), checked
        // against the lane's node; on a hash collision the next lower lane of
        // the slot is tried.
        int pred = -1, hpred = -1;
        if (ntick > 1) {
            const int last0 = 63 - __clzll((long long)gm);  // first lane of the last tick
            L.hmask[2 * l] = 0ull;
            L.hmask[2 * l + 1] = 0ull;
            __syncthreads();
            if (rs && l < last0) atomicOr((unsigned long long *)&L.hmask[head_slot(v)], 1ull << l);
            __syncthreads();
            const int first_l = 63 - __clzll((long long)(gm & le));  // my tick's first lane
            const u64 earlier = first_l > 0 ? ((1ull << first_l) - 1ull) : 0ull;
            u64 m_u = (in && earlier) ? (L.hmask[head_slot(u)] & earlier) : 0ull;
            u64 m_h = (rs && earlier) ? (L.hmask[head_slot(v)] & earlier) : 0ull;
            while (ballot(m_u != 0 || m_h != 0)) {
                const int ju = m_u ? 63 - __clzll((long long)m_u) : l;
                const int jh = m_h ? 63 - __clzll((long long)m_h) : l;
                const int32_t vju = __shfl(v, ju);
                const int32_t vjh = __shfl(v, jh);
                if (m_u) {
                    if (vju == u) { pred = ju; m_u = 0; }
                    else m_u &= ~(1ull << ju);
                }
                if (m_h) {
                    if (vjh == v) { hpred = jh; m_h = 0; }
                    else m_h &= ~(1ull << jh);
                }
            }
        }
        // the next batch's reached-set words, in flight while this one commits
        u32 bu2 = 0, bv2 = 0;
        if (GBM) {
            bu2 = v2 >= 0 ? bm_word<GBM>(bm, u2) : 0u;
            bv2 = v2 >= 0 ? bm_word<GBM>(bm, v2) : 0u;
        }
        bool nw = false;  // my run head was reached first in this batch
        // tick of the latest lane I depend on (-1: none)
        const int dj = pred > hpred ? pred : hpred;
        const int dtk = dj >= 0 ? __popcll(gm & ((2ull << dj) - 1ull)) - 1 : -1;
        // state of my head node after my tick, published by run heads
        u32 pub_h = kHInf;
        u64 pub_S = 0;
        // ---- segments: maximal runs of ticks that read nothing committed inside them
        int ta = 0;
        while (ta < ntick && !done) {
            const u64 br = ballot(in && tid > ta && dtk >= ta);
            const int tb = br ? rl32(tid, __ffsll((long long)br) - 1) : ntick;
            const bool act = in && tid >= ta && tid < tb;
            // tail state: published by an earlier tick of this batch, else batch start
            const bool fu = act && pred >= 0;
            // (the tag test is implied by the bitmap; it keeps the whole loaded
            // word live, so that no register of an in-flight load is reused)
            const bool hub_u = u < H.K;
            u32 h_u = !rt ? kHInf : hub_u ? lhu : ((u32)thu == P.tag) ? ((u32)(thu >> 32) & 0xFFFFu) : kHInf;
            u64 s_u = hub_u ? lsu : su;
            // head state before my tick, likewise
            const bool fh = act && rs && hpred >= 0;
            const bool hub_v = v < H.K;
            u32 cur_h = !hr ? kHInf : hub_v ? lhv : ((u32)thv == P.tag) ? ((u32)(thv >> 32) & 0xFFFFu) : kHInf;
            u64 cur_S = hub_v ? lsv : sv;
            if (ballot(fu || fh)) {
                const int src_u = fu ? pred : l, src_h = fh ? hpred : l;
                const u32 ph_u = (u32)__shfl((int)pub_h, src_u);
                const u64 pS_u = shfl64(pub_S, src_u);
                const u32 ph_h = (u32)__shfl((int)pub_h, src_h);
                const u64 pS_h = shfl64(pub_S, src_h);
                if (fu) { h_u = ph_u; s_u = pS_u; }
                if (fh) { cur_h = ph_h; cur_S = pS_h; }
            }
            const bool reached = act && h_u != kHInf;
            if (!ballot(reached)) {
                if (act && rs) { pub_h = cur_h; pub_S = cur_S; }
                ta = tb;
                continue;
            }
            if (ballot(reached && h_u + 1 >= kHInf)) { o.flags |= REC_HOPS_LIMIT; return; }
            const u32 cand = reached ? h_u + 1 : kBig;
            const u64 am = ballot(act);
            const u64 rsm = ballot(act && rs);
            u32 d;
            u64 c = 0;
            bool tight, lead;
            const bool single = (rsm == am);
            if (single) {
                d = cand;
                tight = reached;
                c = s_u;
                lead = reached;
            } else {
                // runs of several edges: min and exact 96-bit sum through LDS
                if (act && rs) { L.rmin[l] = kBig; L.rlo[l] = 0ull; L.rhi[l] = 0ull; }
                __syncthreads();
                if (reached) atomicMin(&L.rmin[rsl], cand);
                __syncthreads();
                d = act ? L.rmin[rsl] : kBig;
                tight = reached && (P.level ? cand == d : true);
                if (tight) {
                    atomicAdd((unsigned long long *)&L.rlo[rsl], (unsigned long long)(s_u & 0xFFFFFFFFull));
                    atomicAdd((unsigned long long *)&L.rhi[rsl], (unsigned long long)(s_u >> 32));
                }
                __syncthreads();
                lead = act && rs && d != kBig;
                if (lead) {
                    const u64 lo = L.rlo[rsl], hi = L.rhi[rsl];
                    if (hi >> 32) c = kUMax;
                    else { const u64 x = hi << 32; c = x + lo; if (c < x) c = kUMax; }
                }
            }
            // run heads decide
            bool ok = false;
            u32 nh2 = 0;
            u64 nS = 0;
            if (lead) ok = head_commit(opt, cur_h != kHInf, cur_h, cur_S, d, c, v, P.z, zh, &nh2, &nS);
            // fm/sfm/pfm stop at the tick where z is first reached: later ticks
            // of the segment are dropped
            int cut = tb;
            if (opt != OPT_SH) {
                const u64 zm = ballot(ok && v == P.z);
                if (zm) cut = rl32(tid, __ffsll((long long)zm) - 1) + 1;
            }
            const bool keep = tid < cut;
            ok = ok && keep;
            nw = nw || (ok && cur_h == kHInf);
            if (ok) {
                if (v < H.K) { H.h[v] = nh2; H.s[v] = nS; }
                else {
                    Fp[2 * (int64_t)v] = (u64)P.tag | ((u64)nh2 << 32);
                    Fp[2 * (int64_t)v + 1] = nS;
                }
                rch_set<GBM>(bm, v);
            }
            if (SINGLE) {
                // first arrivals: the list of reached nodes, and the hops
                // committed there (fm / sfm / pfm)
                const bool fa = ok && cur_h == kHInf;
                const u64 fm_ = ballot(fa);
                if (fa) {
                    if (FM == FWD_DIST && opt != OPT_SH) Np[v] = (u64)nh2 + 1ull;
                    if (FM == FWD_RTB) {
                        Tp[2 * (int64_t)v] = (u64)(u32)t | ((u64)nh2 << 32);
                        Tp[2 * (int64_t)v + 1] = nS;
                    }
                    Tch[o.reached_n + mbcnt(fm_)] = v;
                }
                o.reached_n += __popcll(fm_);
            }
            if (act && rs) { pub_h = ok ? nh2 : cur_h; pub_S = ok ? nS : cur_S; }
            const u64 zm = ballot(ok && v == P.z);
            if (zm) {
                const int zl = __ffsll((long long)zm) - 1;
                const u32 zh_new = (u32)rl32((int)nh2, zl);
                const int32_t zt = rl32(t, zl);
                if (opt == OPT_SH) { if (zh_new < zh) o.t_arr = zt; }
                else o.t_arr = zt;
                zh = zh_new;
                zS = rl64(nS, zl);
                zhit = true;
            }
            // arcs of the segment
            const bool okr = single ? ok : (__shfl((int)ok, rsl) != 0);
            const bool rec = tight && okr && keep && FM != FWD_DIST;
            const u64 m = ballot(rec);
            if (m) {
                if (!arc_room(a, S, o, o.arcs + __popcll(m))) { o.flags |= REC_ARCS_LIMIT; return; }
                if (rec) put_arc(S, o.arcs + mbcnt(m), v, t, (u32)(b0 + l), u, s_u, h_u, d);
                o.arcs += __popcll(m);
            }
            if (zhit && opt != OPT_SH) {
                done = true;
                const u64 after = ballot(in && tid >= cut);
                o.swept = b0 + (after ? (__ffsll((long long)after) - 1) : nbat) - P.lo;
            }
            ta = tb;
        }
        if (!done) o.swept = (b0 + nbat) - P.lo;
        if (GBM && !done) {
            // the next batch's words were loaded before this batch's commits:
            // the nodes it reached first
            u64 mn = ballot(nw);
            pu = false; pv = false;
            while (mn) {
                const int j = __ffsll((long long)mn) - 1;
                mn &= mn - 1;
                const int32_t w = rl32(v, j);
                pu = pu || u2 == w;
                pv = pv || v2 == w;
            }
            bu = bu2; bv = bv2;
            pref = true;
        }
        __syncthreads();
        b0 += nbat;
        t = t2; u = u2; v = v2; tnext = tn2;
    }
    o.reached = zh != kHInf;
    o.zh = zh;
    o.zS = zS;
}

// element j of a per-slice register array (j is wave-uniform)
__device__ __forceinline__ u64 pick4(const u64 *m, int j) {
    u64 r = m[0];
#pragma unroll
    for (int i = 1; i < kE; ++i) if (j == i) r = m[i];
    return r;
}

// ------------------------------------------------------------ reverse sweep

struct RevCtx {
    u64 sigma;
    u32 dsh;
    int64_t touched_n;
    int64_t edges_n;   // arcs with a non-zero dependency (touched temporal edges)
    bool ovf;
};

// alive set: nodes with a non-zero dependency accumulator for this pair
// (the reached set's bitmap, emptied before the reverse)
template <bool GBM>
__device__ __forceinline__ bool alive_test(const u32 *bm, int32_t v) { return rch_test<GBM>(bm, v); }
template <bool GBM>
__device__ __forceinline__ void alive_set(u32 *bm, int32_t v) { rch_set<GBM>(bm, v); }

__device__ __forceinline__ void rev_contrib(KArgs &a, const Pair &P, const Slab &S,
                                            RevCtx &X, bool act, u64 B, u64 tc, int32_t v, u32 k) {
    u64 *const Np = S.N();
    int32_t *const Tch = S.touched();
    // N(arc) = tail count * B(head); N(v) += N(arc); f(e) = N(arc) / sigma
    bool first = false, wrap = false;
    if (act && B) {
        u64 na = tc * B;
        if (v != P.s && v != P.z) {
            u64 old = atomicAdd((unsigned long long *)&Np[v], (unsigned long long)na);
            first = (old == 0);
            wrap = (old + na < old);
        }
        if (P.req && P.req->Esum) {
            double fe = (double)na / (double)X.sigma;
            atomicAdd(&P.req->Esum[k], fe);
        }
        if (a.edge_f) a.edge_f[P.qout * a.g.m + k] = (double)na / (double)X.sigma;
    }
    if (ballot(wrap)) X.ovf = true;
    X.edges_n += __popcll(ballot(act && B != 0));
    u64 m = ballot(first);
    if (m) {
        int64_t pos = X.touched_n + mbcnt(m);
        if (first) Tch[pos] = v;
        X.touched_n += __popcll(m);
    }
}

__device__ __forceinline__ u64 head_B(const Pair &P, const RevCtx &X, int32_t v, u32 hl, bool valid,
                                      u32 lvl, u64 acc) {
    if (v == P.z) return (P.opt == OPT_SH) ? (hl == X.dsh ? 1ull : 0ull) : 1ull;
    if (!valid) return 0;
    if (P.level && lvl != hl) return 0;
    return acc;
}

// a tick with more arcs than one batch: heads first (all read state older
// than the tick), then level resets and additions at the tails
template <bool GBM>
__device__ void rev_long_tick(KArgs &a, const Pair &P, const Slab &S, u32 *bm, RevCtx &X,
                              int64_t a0, int64_t a1) {
    u64 *const Rp = S.R();
    u64 *const XSp = S.XS();
    const int l = lane_id();
    for (int64_t sb = a0; sb < a1; sb += kWave) {
        int64_t i = sb + l;
        bool inr = i < a1;
        const ArcP ap = arc_at(S, inr ? i : a0);
        u64 mm = inr ? *ap.m : 0;
        int32_t v = (int32_t)(u32)mm;
        bool act = inr && (v == P.z || alive_test<GBM>(bm, v));
        u64 B = 0, tc = 0;
        u32 k = 0;
        if (act) {
            u64 x0 = ap.x[0];
            tc = ap.x[1];
            u32 hl = (u32)(ap.x[2] >> 16) & 0xFFFFu;
            k = (u32)x0;
            bool valid = false;
            u32 lvl = 0;
            u64 acc = 0;
            if (v != P.z) {
                u64 th = ld_agent(&Rp[2 * (int64_t)v]);
                if ((u32)th == P.rtag) { valid = true; lvl = (u32)(th >> 32) & 0xFFFFu; acc = ld_agent(&Rp[2 * (int64_t)v + 1]); }
            }
            B = head_B(P, X, v, hl, valid, lvl, acc);
        }
        if (inr) XSp[i - a0] = B;
        rev_contrib(a, P, S, X, act, B, tc, v, k);
    }
    __syncthreads();
    for (int64_t sb = a0; sb < a1; sb += kWave) {
        int64_t i = sb + l;
        if (i >= a1) continue;
        u64 B = XSp[i - a0];
        if (!B) continue;
        const u64 *xp = arc_x(S, i);
        int32_t u = (int32_t)(xp[0] >> 32);
        u32 tl = (u32)xp[2] & 0xFFFFu;
        u32 want = P.level ? tl : 0u;
        u64 th = ld_agent(&Rp[2 * (int64_t)u]);
        if ((u32)th != P.rtag || ((u32)(th >> 32) & 0xFFFFu) != want) {
            Rp[2 * (int64_t)u] = (u64)P.rtag | ((u64)want << 32);
            Rp[2 * (int64_t)u + 1] = 0;
        }
    }
    __syncthreads();
    bool full = false;
    for (int64_t sb = a0; sb < a1; sb += kWave) {
        int64_t i = sb + l;
        if (i >= a1) continue;
        u64 B = XSp[i - a0];
        if (!B) continue;
        int32_t u = (int32_t)(arc_x(S, i)[0] >> 32);
        atomicAdd((unsigned long long *)&Rp[2 * (int64_t)u + 1], (unsigned long long)B);
        alive_set<GBM>(bm, u);
    }
    __syncthreads();
}

template <bool GBM>
__device__ void reverse(KArgs &a, const Pair &P, const Slab &S, u32 *bm, int64_t bmw, RevLds &L,
                        u32 &stamp, int64_t narcs, RevCtx &X) {
    u64 *const Rp = S.R();
    const int l = lane_id();
    // the alive set starts empty
    if (GBM) {
        uint4 *w4 = reinterpret_cast<uint4 *>(bm);
        for (int64_t w = l; w < bmw; w += kWave) w4[w] = make_uint4(0u, 0u, 0u, 0u);
    } else {
        for (int64_t w = l; w < bmw; w += kWave) bm[w] = 0;
    }
    __syncthreads();
    int64_t ac = narcs;
    while (ac > 0) {
        const int nb = ac < kC ? (int)ac : kC;
        const int64_t blo = ac - nb;
        int32_t vv[kE], tt[kE];
        bool in[kE], al[kE];
        bool any = false;
#pragma unroll
        for (int j = 0; j < kE; ++j) {
            int off = j * kWave + l;
            in[j] = off < nb;
            u64 mm = in[j] ? (*arc_m(S, blo + off)) : 0;
            vv[j] = (int32_t)(u32)mm;
            tt[j] = in[j] ? (int32_t)(mm >> 32) : INT32_MIN;
            al[j] = in[j] && (vv[j] == P.z || alive_test<GBM>(bm, vv[j]));
            if (ballot(al[j])) any = true;
        }
        // no arc of this batch can carry a dependency: nothing to do
        if (!any) { ac = blo; continue; }
        // cut at a tick boundary at the low end
        int cut = 0;
        if (blo > 0) {
            int32_t t_first = rl32(tt[0], 0);
            int32_t t_before = (int32_t)((*arc_m(S, blo - 1)) >> 32);
            if (t_before == t_first) {
                int firstdiff = -1;
#pragma unroll
                for (int j = 0; j < kE; ++j) {
                    u64 m = ballot(in[j] && tt[j] != t_first);
                    if (firstdiff < 0 && m) firstdiff = j * kWave + (__ffsll((long long)m) - 1);
                }
                if (firstdiff < 0) {
                    int64_t a0 = 0;
                    for (int64_t i = blo - kWave; ; i -= kWave) {
                        int64_t idx = i + l;
                        bool okk = idx >= 0 && idx < blo;
                        bool diff = okk && (int32_t)((*arc_m(S, idx)) >> 32) != t_first;
                        u64 m = ballot(diff);
                        if (m) { a0 = i + (63 - __clzll((long long)m)) + 1; break; }
                        if (i <= 0) { a0 = 0; break; }
                    }
                    rev_long_tick<GBM>(a, P, S, bm, X, a0, ac);
                    ac = a0;
                    continue;
                }
                cut = firstdiff;
            }
        }
        // arcs of the batch: tails and counts
        u64 tc[kE];
        u32 kk[kE], tl[kE], hl[kE];
        int32_t uu[kE];
        u64 gm[kE];
        bool hval[kE], tval[kE];
        u32 hlvl[kE], tlvl[kE];
        u64 hacc[kE], tacc[kE];
#pragma unroll
        for (int j = 0; j < kE; ++j) {
            int off = j * kWave + l;
            in[j] = in[j] && off >= cut;
            al[j] = al[j] && in[j];
            int32_t tp = __shfl_up(tt[j], 1);
            if (l == 0) tp = j > 0 ? rl32(tt[j - 1], kWave - 1) : INT32_MIN;
            gm[j] = ballot(in[j] && (off == cut || tt[j] != tp));
            const u64 *xp = arc_x(S, in[j] ? blo + off : blo);
            u64 x0 = in[j] ? xp[0] : 0;
            tc[j] = in[j] ? xp[1] : 0;
            u64 x2 = in[j] ? xp[2] : 0;
            kk[j] = (u32)x0;
            uu[j] = (int32_t)(x0 >> 32);
            tl[j] = (u32)x2 & 0xFFFFu;
            hl[j] = (u32)(x2 >> 16) & 0xFFFFu;
            hval[j] = false; hlvl[j] = 0; hacc[j] = 0;
            tval[j] = false; tlvl[j] = 0; tacc[j] = 0;
            if (al[j] && vv[j] != P.z) {
                u64 th = ld_agent(&Rp[2 * (int64_t)vv[j]]);
                if ((u32)th == P.rtag) { hval[j] = true; hlvl[j] = (u32)(th >> 32) & 0xFFFFu; hacc[j] = ld_agent(&Rp[2 * (int64_t)vv[j] + 1]); }
            }
            if (in[j] && alive_test<GBM>(bm, uu[j])) {
                u64 th = ld_agent(&Rp[2 * (int64_t)uu[j]]);
                if ((u32)th == P.rtag) { tval[j] = true; tlvl[j] = (u32)(th >> 32) & 0xFFFFu; tacc[j] = ld_agent(&Rp[2 * (int64_t)uu[j] + 1]); }
            }
        }
        stamp += 1;
        bool used = false;
        __syncthreads();
        int ge = nb;
        while (ge > cut) {
            int gs = cut;
            {
                int pos = ge - 1;
                for (int j = pos >> 6; j >= 0; --j) {
                    u64 m = pick4(gm, j);
                    int b = (j == (pos >> 6)) ? (pos & 63) : 63;
                    m &= (b == 63) ? kUMax : ((2ull << b) - 1ull);
                    if (m) { gs = j * kWave + 63 - __clzll((long long)m); break; }
                }
            }
            const int jlo = gs >> 6, jhi = (ge - 1) >> 6;
            u64 Bv[kE];
            bool anyB = false;
#pragma unroll
            for (int j = 0; j < kE; ++j) {
                Bv[j] = 0;
                if (j < jlo || j > jhi) continue;
                int off = j * kWave + l;
                bool inr = off >= gs && off < ge;
                bool act = false;
                if (inr) {
                    bool valid = hval[j];
                    u32 lvl = hlvl[j];
                    u64 acc = hacc[j];
                    act = al[j];
                    if (used && vv[j] != P.z) {
                        int sl = tab_find(L.tb_key, stamp, (u32)vv[j]);
                        if (sl >= 0) { u32 x = L.tb_lvl[sl]; valid = (x >> 31) != 0; lvl = x & 0xFFFFu; acc = L.tb_acc[sl]; act = true; }
                    }
                    if (act) Bv[j] = head_B(P, X, vv[j], hl[j], valid, lvl, acc);
                }
                if (ballot(act)) rev_contrib(a, P, S, X, act, Bv[j], tc[j], vv[j], kk[j]);
                if (ballot(Bv[j] != 0)) anyB = true;
            }
            if (anyB) {
                used = true;
                int tsl[kE];
#pragma unroll
                for (int j = 0; j < kE; ++j) {
                    tsl[j] = -1;
                    if (j < jlo || j > jhi) continue;
                    if (Bv[j]) {
                        int fresh;
                        tsl[j] = tab_insert(L.tb_key, stamp, (u32)uu[j], &fresh);
                        if (fresh) {
                            L.tb_lvl[tsl[j]] = tval[j] ? ((tlvl[j] & 0xFFFFu) | 0x80000000u) : 0u;
                            L.tb_acc[tsl[j]] = tval[j] ? tacc[j] : 0ull;
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < kE; ++j) {
                    if (tsl[j] < 0) continue;
                    u32 want = P.level ? tl[j] : 0u;
                    u32 x = L.tb_lvl[tsl[j]];
                    if (!(x >> 31) || (x & 0xFFFFu) != want) {
                        L.tb_lvl[tsl[j]] = want | 0x80000000u;
                        L.tb_acc[tsl[j]] = 0;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < kE; ++j) {
                    if (tsl[j] < 0) continue;
                    atomicAdd((unsigned long long *)&L.tb_acc[tsl[j]], (unsigned long long)Bv[j]);
                    alive_set<GBM>(bm, uu[j]);
                }
                __syncthreads();
            }
            ge = gs;
        }
        if (used) {
            for (int sl = l; sl < kFwN; sl += kWave) {
                u64 key = L.tb_key[sl];
                if ((u32)(key >> 32) != stamp) continue;
                u32 node = (u32)key;
                u32 x = L.tb_lvl[sl];
                Rp[2 * (int64_t)node] = (u64)P.rtag | ((u64)(x & 0xFFFFu) << 32);
                Rp[2 * (int64_t)node + 1] = L.tb_acc[sl];
            }
        }
        __syncthreads();
        ac = blo + cut;
    }
}

// ------------------------------------------------------------ the kernel

// SINGLE (the distance kernel): slots are single sources, no target
template <bool SINGLE = false, class A>
__device__ void resolve_pair(A &a, int64_t slot, Pair &P) {
    // a retry launch names the original launch slots through pq
    const int64_t q = a.pq ? (int64_t)a.pq[slot] : slot;
    int r = 0;
    while (r + 1 < a.nreq && q >= a.reqs[r + 1].qoff) ++r;
    const DevReq &R = a.reqs[r];
    P.req = &R;
    P.opt = R.opt; P.t0 = R.t0; P.t1 = R.t1; P.c = R.c;
    P.q = q;
    P.qout = q;
    P.lam = 0;
    const int64_t i = q - R.qoff + R.base;
    u64 pstream = (u64)R.stream;
    P.trk_i = (u64)i;
    if (a.ps) {
        P.g = a.pg ? a.pg[q] : 0;
        P.s = a.ps[q];
        P.z = SINGLE ? -1 : a.pz[q];
    } else {
        int64_t idx;
        if (R.graph >= 0) { P.g = R.graph; idx = i; }
        else { P.g = (int32_t)(i / R.per_graph); idx = i % R.per_graph; }
        int32_t noff = a.g.seg_noff[P.g];
        int32_t ng = a.g.seg_noff[P.g + 1] - noff;
        u64 st = (u64)R.stream + (u64)STREAMS_PER_GRAPH * (u64)P.g;
        pstream = st;
        P.trk_i = (u64)idx;
        u64 s = __umul64hi(rng_word(R.seed, st, (u64)idx, 0), (u64)ng);
        u64 zp = __umul64hi(rng_word(R.seed, st, (u64)idx, 1), (u64)(ng - 1));
        // pairs are drawn over input ids, then mapped to internal ids
        P.s = a.g.perm[noff + (int32_t)s] - noff;
        P.z = SINGLE ? -1 : a.g.perm[noff + (int32_t)(zp + (zp >= s ? 1 : 0))] - noff;
        if (R.c > 0) P.lam = rng_word(R.seed, (u64)STREAM_RADE + (u64)STREAMS_PER_GRAPH * (u64)P.g, (u64)idx, 0);
    }
    P.noff = a.g.seg_noff[P.g];
    P.ng = a.g.seg_noff[P.g + 1] - P.noff;
    P.elo = a.g.seg_eoff[P.g];
    P.ehi = a.g.seg_eoff[P.g + 1];
    P.level = (P.opt == OPT_SH || P.opt == OPT_SFM);
    P.single = SINGLE;
    P.trk_key = sm_mix(R.seed + (kStreamTrk + pstream + 1ull) * 0x9E3779B97F4A7C15ull);
}

// Distances from a single source after its forward sweep: every node the
// sweep reached (other than the source; the forward lists them in
// the slab's touched list at their first arrival) adds one to the bin of its distance.
// sh: fewest hops over all arrivals (the final hop state); fm, sfm and pfm:
// the hops committed at the first arrival, which the forward keeps in N as
// hops + 1 (N must be zero again for the next slot, so it is cleared here,
// also when the sweep stopped at the hops limit and nothing is counted).
constexpr int kDistBins = 2 * kFwN;  // u32 bins in LDS, over the reverse table's keys
static_assert(kDistBins * 4 <= (int)sizeof(u64) * kFwN, "distance bins exceed the table");

__device__ void distance_hist(const Pair &P, const Slab &S, const Hub &H, u32 *lh, int64_t nreached, bool count) {
    u64 *const Np = S.N();
    int32_t *const Tch = S.touched();
    u64 *const Fp = S.F();
    const int l = lane_id();
    const DevReq *R = P.req;
    const u32 last = (u32)R->hist_len - 1u;
    const bool first = P.opt != OPT_SH;
    for (int i = l; i < kDistBins; i += kWave) lh[i] = 0u;
    __syncthreads();
    u32 dmax = 0;
    for (int64_t i = l; i < nreached; i += kWave) {
        const int32_t v = Tch[i];
        u32 d;
        if (first) {
            d = (u32)(Np[v] - 1ull);
            Np[v] = 0ull;
        } else {
            d = v < H.K ? H.h[v] : (u32)(Fp[2 * (int64_t)v] >> 32) & 0xFFFFu;
        }
        if (count) {
            const u32 b = d < last ? d : last;
            if (b < (u32)kDistBins) atomicAdd(&lh[b], 1u);
            else atomicAdd((unsigned long long *)&R->hist[b], 1ull);
            dmax = d > dmax ? d : dmax;
        }
    }
    __syncthreads();
    if (!count) return;
    for (u32 i = (u32)l; i < (u32)kDistBins && i <= last; i += kWave)
        if (lh[i]) atomicAdd((unsigned long long *)&R->hist[i], (unsigned long long)lh[i]);
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const u32 x = (u32)__shfl_xor((int)dmax, o);
        dmax = x > dmax ? x : dmax;
    }
    if (l == 0 && dmax) atomicMax((unsigned long long *)&R->hist[last + 1u], (unsigned long long)dmax);
    __syncthreads();
}

// The TRK estimator (appendix on other estimators): one optimal walk of the
// pair, drawn backwards from z with the probability 1/sigma_sz, and
// f(v) = the number of its internal visits of v (v not s or z), f(e) = its
// uses of e.  Each step draws one recorded arc, with the probability of its
// tail count among the candidates:
//  - first step: the arcs into z's terminal appearances (sh: those at z's
//    fewest hops; fm, sfm, pfm: those at z's first arrival);
//  - then, after an arc with tail x at level L and time t: the arcs into the
//    appearances of x before t (sh, sfm: at level L; pfm: x's first
//    arrival; fm: all of them), and for fm at x = s the origin (weight 1,
//    first); for sh, sfm and pfm the walk ends at x = s.
// An arc's tail count is the number of optimal prefixes of its tail node
// that it extends, so the first step picks (z, t_z) with probability
// sigma(z, t_z) / sigma_sz and each later step picks the predecessor
// appearance and its arc together, as the paper's backward sampler does.
// The draw of step j is r = floor(w * W / 2^64) with w the SplitMix64 output
// (pair index * 2^16 + j + 1) of the pair's path stream and W the candidates'
// total; the arc taken is the first, in arc order (time, then input head and
// tail ids), whose running total exceeds r.  Each step's total must equal
// the count it stands for (sigma_sz first, then the tail count of the arc
// taken); returns false where it does not.
__device__ bool trk_walk(KArgs &a, const Pair &P, const Slab &S, int64_t narcs, u32 zh, int32_t t_arr,
                         u64 sigma, RevCtx &X) {
    u64 *const Np = S.N();
    int32_t *const Tch = S.touched();
    const int l = lane_id();
    const DevReq *R = P.req;
    int32_t node = P.z;
    u32 lvl = zh;
    int32_t tmax = INT32_MAX;
    int64_t hi = narcs;
    bool term = true;
    u64 expect = sigma;
    for (u32 step = 0;; ++step) {
        const bool origin = !term && node == P.s;  // fm only: the walk may start here
        // pass 1: total weight of the candidates
        u64 part = 0;
        for (int64_t b = 0; b < hi; b += kWave) {
            const int64_t i = b + l;
            if (i >= hi) continue;
            const ArcP ap = arc_at(S, i);
            const u64 mm = *ap.m;
            if ((int32_t)(u32)mm != node) continue;
            const int32_t ti = (int32_t)(mm >> 32);
            const u32 hl = (u32)(ap.x[2] >> 16) & 0xFFFFu;
            bool c;
            if (term) c = P.opt == OPT_SH ? hl == lvl : ti == t_arr;
            else c = ti < tmax && (!P.level || hl == lvl);
            if (c) part = sat_add(part, ap.x[1]);
        }
        for (int o = kWave / 2; o > 0; o >>= 1) part = sat_add(part, shfl64(part, l ^ o));
        u64 W = uni64(part);
        if (origin) W = sat_add(W, 1ull);
        if (W != expect || W == 0 || W == kUMax) return false;
        const u64 w = sm_mix(P.trk_key + ((P.trk_i << 16) + (u64)step + 1ull) * 0x9E3779B97F4A7C15ull);
        const u64 r = __umul64hi(w, W);
        if (origin && r < 1ull) return true;  // the walk starts at the origin
        // pass 2: the first candidate whose running total exceeds r
        u64 carry = origin ? 1ull : 0ull;
        int64_t pick = -1;
        for (int64_t b = 0; b < hi && pick < 0; b += kWave) {
            const int64_t i = b + l;
            u64 wt = 0;
            if (i < hi) {
                const ArcP ap = arc_at(S, i);
                const u64 mm = *ap.m;
                if ((int32_t)(u32)mm == node) {
                    const int32_t ti = (int32_t)(mm >> 32);
                    const u32 hl = (u32)(ap.x[2] >> 16) & 0xFFFFu;
                    bool c;
                    if (term) c = P.opt == OPT_SH ? hl == lvl : ti == t_arr;
                    else c = ti < tmax && (!P.level || hl == lvl);
                    if (c) wt = ap.x[1];
                }
            }
            // inclusive scan of the weights over the wave (no wrap: the
            // total is below 2^64 - 1)
            u64 x = wt;
            for (int o = 1; o < kWave; o <<= 1) {
                const u32 lo = (u32)__shfl_up((int)(u32)x, o), hi32 = (u32)__shfl_up((int)(u32)(x >> 32), o);
                const u64 y = ((u64)hi32 << 32) | lo;
                if (l >= o) x += y;
            }
            const u64 hit = ballot(wt != 0 && carry + x > r);
            if (hit) pick = b + (__ffsll((long long)hit) - 1);
            else carry += rl64(x, kWave - 1);
        }
        if (pick < 0) return false;
        const ArcP pp = arc_at(S, pick);
        const u64 x0 = pp.x[0];
        const int32_t k = (int32_t)(u32)x0;           // stream index of the edge
        const int32_t tail = (int32_t)(x0 >> 32);
        const u32 tl = (u32)pp.x[2] & 0xFFFFu;
        const int32_t tp = (int32_t)(*pp.m >> 32);
        const u64 tcp = pp.x[1];
        // visit counts in the slab's N (zero between pairs) and the list of
        // the distinct internal nodes, as the reverse sweep leaves them
        if (tail != P.s && tail != P.z) {
            const u64 old = Np[tail];  // every lane reads the same word
            if (l == 0) {
                Np[tail] = old + 1ull;
                if (old == 0ull) Tch[X.touched_n] = tail;
            }
            if (old == 0ull) X.touched_n += 1;
        }
        if (l == 0) {
            if (R->Esum) atomicAdd(&R->Esum[k], 1.0);
            if (a.edge_f) a.edge_f[P.qout * a.g.m + (int64_t)(u32)k] += 1.0;
        }
        __syncthreads();  // the visit count is read again if the walk comes back
        X.edges_n += 1;
        if (tail == P.s && P.opt != OPT_FM) return true;  // the origin
        node = tail;
        lvl = tl;
        tmax = tp;
        hi = pick;
        term = false;
        expect = tcp;
    }
}

// The RTB estimator (appendix on other estimators): for a sampled source s,
// f(v|s) = (1/(n-1)) * sum over targets z != s of sigma_sz(v) / sigma_sz.
// After a forward sweep of s to the window's end with its arcs recorded, the
// reverse walks the arcs newest first, one tick at a time, in double
// precision: the value of a head appearance (v, t) is
//   C(v, t) = (continuations of (v, t), the tail state of v at its level)
//           + 1 / sigma_sv if (v, t) is one of v's terminal appearances
// (sh: those at v's fewest hops; fm, sfm, pfm: its first arrival), i.e. the
// sum over targets z of (optimal suffixes from (v, t) to z) / sigma_sz.
// N(v) gains (tail count) * (continuations only: v as the target is not an
// internal node), f(e) = (tail count) * C(head) / (n - 1), and C(head) flows
// into the tail's state; level resets as in the pair reverse.  The origin's
// value must come out as the number of reached targets.  Returns false if
// a count on the way saturated.
__device__ bool rev_rtb(KArgs &a, const Pair &P, const Slab &S, int64_t narcs, RevCtx &X) {
    u64 *const Rp = S.R();
    u64 *const XSp = S.XS();
    u64 *const Tp = S.T();
    u64 *const Np = S.N();
    int32_t *const Tch = S.touched();
    const int l = lane_id();
    const DevReq *R = P.req;
    const double n1 = (double)(P.ng - 1);
    bool bad = false;
    int64_t ac = narcs;
    while (ac > 0) {
        // the tick [a0, ac) of the newest arcs left
        const int32_t th = (int32_t)((*arc_m(S, ac - 1)) >> 32);
        int64_t a0 = 0;
        for (int64_t i0 = ac - kWave;; i0 -= kWave) {
            const int64_t i = i0 + l;
            const bool diff = i >= 0 && i < ac && (int32_t)((*arc_m(S, i)) >> 32) != th;
            const u64 m = ballot(diff);
            if (m) { a0 = i0 + (63 - __clzll((long long)m)) + 1; break; }
            if (i0 <= 0) { a0 = 0; break; }
        }
        // heads: their values (state older than the tick), N(v), f(e)
        for (int64_t sb = a0; sb < ac; sb += kWave) {
            const int64_t i = sb + l;
            bool first = false, nz = false;
            int32_t v = 0;
            if (i < ac) {
                const ArcP ap = arc_at(S, i);
                const u64 mm = *ap.m;
                v = (int32_t)(u32)mm;
                const int32_t t = (int32_t)(mm >> 32);
                const u64 x0 = ap.x[0];
                const u32 k = (u32)x0;
                const u64 tc = ap.x[1];
                const u32 hl = (u32)(ap.x[2] >> 16) & 0xFFFFu;
                if (tc == kUMax) bad = true;
                double thru = 0.0;
                const u64 tw = ld_agent(&Rp[2 * (int64_t)v]);
                if ((u32)tw == P.rtag && (!P.level || ((u32)(tw >> 32) & 0xFFFFu) == hl))
                    thru = __longlong_as_double((long long)ld_agent(&Rp[2 * (int64_t)v + 1]));
                double C = thru;
                if (v != P.s) {
                    const u64 fa = Tp[2 * (int64_t)v];
                    const bool term = P.opt == OPT_SH ? ((u32)(fa >> 32) & 0xFFFFu) == hl : (int32_t)(u32)fa == t;
                    if (term) {
                        const u64 sg = Tp[2 * (int64_t)v + 1];
                        if (sg == kUMax) bad = true;
                        C += 1.0 / (double)sg;
                    }
                }
                XSp[i - a0] = (u64)__double_as_longlong(C);
                if (v != P.s && thru != 0.0) {
                    const double old = atomicAdd(reinterpret_cast<double *>(&Np[v]), (double)tc * thru);
                    first = old == 0.0;
                }
                nz = C != 0.0;
                if (nz) {
                    const double fe = (double)tc * C / n1;
                    if (R->Esum) atomicAdd(&R->Esum[k], fe);
                    if (a.edge_f) a.edge_f[P.qout * a.g.m + k] = fe;
                }
            }
            X.edges_n += __popcll(ballot(nz));
            const u64 m = ballot(first);
            if (first) Tch[X.touched_n + mbcnt(m)] = v;
            X.touched_n += __popcll(m);
        }
        __syncthreads();
        // tails: level resets, then the additions
        for (int64_t sb = a0; sb < ac; sb += kWave) {
            const int64_t i = sb + l;
            if (i >= ac) continue;
            if (XSp[i - a0] == 0ull) continue;
            const u64 *xp = arc_x(S, i);
            const int32_t u = (int32_t)(xp[0] >> 32);
            const u32 want = P.level ? ((u32)xp[2] & 0xFFFFu) : 0u;
            const u64 tw = ld_agent(&Rp[2 * (int64_t)u]);
            if ((u32)tw != P.rtag || ((u32)(tw >> 32) & 0xFFFFu) != want) {
                Rp[2 * (int64_t)u] = (u64)P.rtag | ((u64)want << 32);
                Rp[2 * (int64_t)u + 1] = 0ull;
            }
        }
        __syncthreads();
        for (int64_t sb = a0; sb < ac; sb += kWave) {
            const int64_t i = sb + l;
            if (i >= ac) continue;
            const u64 cb = XSp[i - a0];
            if (cb == 0ull) continue;
            const int32_t u = (int32_t)(arc_x(S, i)[0] >> 32);
            atomicAdd(reinterpret_cast<double *>(&Rp[2 * (int64_t)u + 1]), __longlong_as_double((long long)cb));
        }
        __syncthreads();
        ac = a0;
    }
    return !ballot(bad);
}

// MODE_PAIRS: pairs, f = N / sigma from the reverse sweep; MODE_DISTANCES:
// every slot is a single source; MODE_TRK: pairs, f = visits of one sampled
// optimal walk.  Each mode is a kernel of its own, so that the pair sweep
// keeps its register allocation.
__device__ __forceinline__ Slab slab_of(int64_t slab, u32 *xtl) {
    Slab S;
    S.id = slab;
    S.xtl = xtl;
    return S;
}

// GBM: the reached set in a bitmap in the slab's global memory (graphs of
// more than 65,536 nodes) instead of in LDS
template <int MODE, bool GBM>
__global__ void __launch_bounds__(64, MANTRA_SWEEP_WPS) k_sweep(LaunchArgs a_arg) {
    constexpr bool RTB = MODE == MODE_RTB;
    constexpr bool SINGLE = MODE == MODE_DISTANCES || RTB;
    constexpr bool TRK = MODE == MODE_TRK;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int l = lane_id();
    const int64_t slab = blockIdx.x;
    (void)a_arg;
    TabLds &tab = *reinterpret_cast<TabLds *>(lds_raw);
    for (int i = l; i < kFwN; i += kWave) { tab.r.tb_key[i] = 0; }
    u32 serial;
    int64_t np;
    {
        KArgs &a = launch_args();
        const u32 *hdr = a.sl.hdr + slab * 4;
        serial = hdr[0];
        np = a.npairs_dev ? *a.npairs_dev : a.npairs;
    }
    u32 stamp = 1;  // reverse table stamps (0 = empty)
    const u64 t_begin = wall_clock64();
    u64 fwd_ticks = 0, rev_ticks = 0;  // time in forward sweeps, in the rest of the pairs
    __syncthreads();
    for (;;) {
        KArgs &a = launch_args();
        const Slab S = slab_of(slab, reinterpret_cast<u32 *>(lds_raw + sizeof(TabLds)));
        // LDS bitmap words, or the 16-byte words of the bitmap in global memory
        const int64_t bmw = GBM ? (a.sl.nmax + 127) / 128 : (a.sl.nmax + 31) / 32;
        constexpr size_t kHead = sizeof(TabLds) + sizeof(u32) * kXtLds;  // tables, chunk table
        u32 *bm = GBM ? reinterpret_cast<u32 *>(a.sl.BM + slab * bmw * 16)
                      : reinterpret_cast<u32 *>(lds_raw + kHead);
        Hub H;
        H.K = a.hub_nodes;
        H.s = reinterpret_cast<u64 *>(lds_raw + kHead + (GBM ? 0 : ((bmw * 4 + 7) & ~7ll)));
        H.h = reinterpret_cast<u32 *>(H.s + H.K);
        u32 qq = 0;
        if (l == 0) qq = atomicAdd(a.work, 1u);
        const int64_t q = a.qbase + (int64_t)(u32)uni((int)qq);
        if (q >= np) break;
        Pair P;
        resolve_pair<SINGLE>(a, q, P);
        // two tags per pair; 0 and 1 never valid (fresh slabs are zero)
        serial += 2;
        if (serial < 2u) serial = 2u;
        P.tag = serial;
        P.rtag = serial + 1u;
        // window: first departure of s, last arrival at z, inside [t0, t1]
        // (a single source: to the end of [t0, t1])
        const int32_t gs_node = P.noff + P.s;
        int64_t o0 = a.g.out_off[gs_node], o1 = a.g.out_off[gs_node + 1];
        int64_t od = wave_lower_bound(a.g.out_t, o0, o1, P.t0);
        bool ok;
        int32_t dep, lin;
        if (SINGLE) {
            ok = od < o1;
            dep = ok ? a.g.out_t[od] : 0;
            lin = P.t1;
            ok = ok && dep <= P.t1;
        } else {
            const int32_t gz_node = P.noff + P.z;
            int64_t i0 = a.g.in_off[gz_node], i1 = a.g.in_off[gz_node + 1];
            int64_t id = wave_upper_bound(a.g.in_t, i0, i1, P.t1) - 1;
            ok = od < o1 && id >= i0;
            dep = ok ? a.g.out_t[od] : 0;
            lin = ok ? a.g.in_t[id] : 0;
            ok = ok && dep <= P.t1 && lin >= P.t0 && lin >= dep;
        }
        FwdOut fo;
        fo.reached = false; fo.zh = kHInf; fo.zS = 0; fo.t_arr = -1; fo.arcs = 0; fo.swept = 0; fo.flags = 0;
        fo.reached_n = 0;
        fo.room = a.sl.cap;
        fo.nch = 0;
        fo.live = fo.dead = 0;
        if (ok) {
            P.lo = wave_lower_bound(a.g.T, P.elo, P.ehi, dep);
            P.hi = wave_upper_bound(a.g.T, P.lo, P.ehi, lin);
            // reset the reached set and the hub hops (unreached: kHInf), seed
            // the origin
            if (GBM) {
                uint4 *w4 = reinterpret_cast<uint4 *>(bm);
                for (int64_t w = l; w < bmw; w += kWave) w4[w] = make_uint4(0u, 0u, 0u, 0u);
            } else {
                for (int64_t w = l; w < bmw; w += kWave) bm[w] = 0;
            }
            for (int i = l; i < H.K; i += kWave) H.h[i] = kHInf;
            __syncthreads();
            if (l == 0) {
                if (P.s < H.K) { H.h[P.s] = 0u; H.s[P.s] = 1ull; }
                else {
                    S.F()[2 * (int64_t)P.s] = (u64)P.tag;  // h = 0
                    S.F()[2 * (int64_t)P.s + 1] = 1ull;
                }
                rch_set<GBM>(bm, P.s);
            }
            __syncthreads();
            const u64 c0 = wall_clock64();
            forward<SINGLE ? (RTB ? FWD_RTB : FWD_DIST) : FWD_PAIR, GBM>(a, P, S, bm, H, tab.f, fo);
            fwd_ticks += wall_clock64() - c0;
            __syncthreads();
            if (MODE == MODE_DISTANCES)
                distance_hist(P, S, H, reinterpret_cast<u32 *>(tab.r.tb_key), fo.reached_n,
                              !(fo.flags & REC_HOPS_LIMIT));
            if (RTB) {
                // sh: the terminal level and sigma are the final state
                for (int64_t i = l; i < fo.reached_n; i += kWave) {
                    const int32_t v = S.touched()[i];
                    const u32 h = v < H.K ? H.h[v] : (u32)(S.F()[2 * (int64_t)v] >> 32) & 0xFFFFu;
                    const u64 sg = v < H.K ? H.s[v] : S.F()[2 * (int64_t)v + 1];
                    if (P.opt == OPT_SH) {
                        S.T()[2 * (int64_t)v] = (u64)h << 32;
                        S.T()[2 * (int64_t)v + 1] = sg;
                    }
                }
            }
            // the reverse table reuses the forward's LDS: empty it
            for (int i = l; i < kFwN; i += kWave) { tab.r.tb_key[i] = 0; }
            stamp = 1;
            __syncthreads();
        }
        const u64 c1 = wall_clock64();
        u32 flags = fo.flags;
        bool reach = ok && fo.reached && !(flags & (REC_HOPS_LIMIT | REC_ARCS_LIMIT));
        u64 sigma = reach ? fo.zS : 0;
        if (reach && sigma == kUMax) flags |= REC_OVERFLOW;
        if (RTB) {
            // a source: sigma counts the targets it reaches
            reach = ok && fo.reached_n > 0 && !(flags & (REC_HOPS_LIMIT | REC_ARCS_LIMIT));
            sigma = reach ? (u64)fo.reached_n : 0;
        }
        bool do_rev = reach && !(flags & REC_OVERFLOW);
        RevCtx X;
        X.sigma = sigma; X.dsh = fo.zh; X.touched_n = 0; X.edges_n = 0; X.ovf = false;
        if (RTB && do_rev) {
            if (!rev_rtb(a, P, S, fo.arcs, X)) {
                // a saturated count: the source is void, its f(e) rows cleared
                flags |= REC_OVERFLOW;
                if (a.edge_f)
                    for (int64_t i = l; i < fo.arcs; i += kWave)
                        a.edge_f[P.qout * a.g.m + (int64_t)(u32)arc_x(S, i)[0]] = 0.0;
            } else {
                // every reached target contributes exactly one to the origin
                const u64 tw = ld_agent(&S.R()[2 * (int64_t)P.s]);
                double bo = 0.0;
                if ((u32)tw == P.rtag && (!P.level || ((u32)(tw >> 32) & 0xFFFFu) == 0u))
                    bo = __longlong_as_double((long long)ld_agent(&S.R()[2 * (int64_t)P.s + 1]));
                const double want = (double)fo.reached_n;
                if (!(fabs(bo - want) <= 1e-9 * want)) flags |= REC_SELFCHECK;
            }
        } else if (TRK && do_rev) {
            // the walk checks the forward's counts at every step: a failure
            // is a broken invariant
            if (!trk_walk(a, P, S, fo.arcs, fo.zh, fo.t_arr, sigma, X)) flags |= REC_SELFCHECK;
        } else if (do_rev) {
            reverse<GBM>(a, P, S, bm, bmw, tab.r, stamp, fo.arcs, X);
            __syncthreads();
            // flow conservation at the origin: B(origin) must equal sigma
            u64 th = ld_agent(&S.R()[2 * (int64_t)P.s]);
            u64 bo = 0;
            if ((u32)th == P.rtag && (!P.level || ((u32)(th >> 32) & 0xFFFFu) == 0u)) bo = ld_agent(&S.R()[2 * (int64_t)P.s + 1]);
            if (bo != sigma) flags |= REC_SELFCHECK;
        }
        if (X.ovf) {
            // an fm visit count wrapped during the reverse sweep: the pair is
            // reported as saturated, so the f(e) it already wrote are cleared
            // (its sums are void: the request fails with MANTRA_E_OVERFLOW)
            flags |= REC_OVERFLOW;
            if (a.edge_f)
                for (int64_t i = l; i < fo.arcs; i += kWave)
                    a.edge_f[P.qout * a.g.m + (int64_t)(u32)arc_x(S, i)[0]] = 0.0;
        }
        // finalize: f(v) = N(v) / sigma into the sums; reset N
        bool accum = do_rev && !(flags & REC_OVERFLOW);
        const DevReq *R = P.req;
        for (int64_t i = l; i < X.touched_n; i += kWave) {
            int32_t v = S.touched()[i];
            u64 nv = atomicExch((unsigned long long *)&S.N()[v], 0ull);
            if (!accum) continue;
            double f = TRK ? (double)nv
                           : RTB ? __longlong_as_double((long long)nv) / (double)(P.ng - 1) : (double)nv / (double)sigma;
            int64_t gv = (int64_t)P.noff + v;
            if (R->Bsum) atomicAdd(&R->Bsum[gv], f);
            if (R->Wsum) { double f2 = f * f; atomicAdd(&R->Wsum[gv], f2); }
            if (R->Rsum) {
                for (int jc = 0; jc < P.c; ++jc) {
                    double x = ((P.lam >> jc) & 1ull) ? -f : f;
                    atomicAdd(&R->Rsum[gv * P.c + jc], x);
                }
            }
            if (a.node_f) a.node_f[P.qout * (int64_t)a.g.n_total + gv] = f;
        }
        // the pair's arcs are read no more: its shared chunks go back
        chunks_free(a, S, fo.nch);
        rev_ticks += wall_clock64() - c1;
        if (l == 0) {
            if (a.rec) {
                int32_t *rr = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(a.rec) + P.qout * 24);
                bool rch = reach;
                rr[0] = rch ? 1 : 0;
                rr[1] = rch ? fo.t_arr : -1;
                rr[2] = (rch && !RTB) ? (int32_t)fo.zh : -1;
                rr[3] = (int32_t)flags;
                *reinterpret_cast<u64 *>(rr + 4) = sigma;
            }
            if (!(flags & REC_ARCS_LIMIT)) {
                atomicAdd((unsigned long long *)&a.stats[0], (unsigned long long)fo.swept);
                atomicAdd((unsigned long long *)&a.stats[1], (unsigned long long)fo.arcs);
            }
            // saturated pairs go to the multiword path when there is one
            const bool defer = MODE == MODE_PAIRS && a.wide && (flags & REC_OVERFLOW) && !(flags & REC_ARCS_LIMIT) &&
                               (a.wide_fm || P.opt != OPT_FM);
            if (defer) {
                const int pos = atomicAdd(&a.wide[0], 1);
                a.wide[1 + pos] = (int32_t)P.q;
            }
            if ((flags & REC_OVERFLOW) && !defer) atomicAdd((unsigned long long *)&a.stats[2], 1ull);
            if (reach) atomicAdd((unsigned long long *)&a.stats[3], 1ull);
            if (flags & REC_HOPS_LIMIT) atomicAdd((unsigned long long *)&a.stats[4], 1ull);
            if (flags & REC_SELFCHECK) atomicAdd((unsigned long long *)&a.stats[6], 1ull);
            atomicAdd((unsigned long long *)&a.stats[7], (unsigned long long)X.touched_n);
            atomicAdd((unsigned long long *)&a.stats[14], (unsigned long long)fo.live);
            atomicAdd((unsigned long long *)&a.stats[15], (unsigned long long)fo.dead);
            atomicAdd((unsigned long long *)&a.stats[8], (unsigned long long)X.edges_n);
            if (R->rstat && !(flags & REC_ARCS_LIMIT)) {
                if ((flags & REC_OVERFLOW) && !defer) atomicAdd((unsigned long long *)&R->rstat[0], 1ull);
                if (reach) atomicAdd((unsigned long long *)&R->rstat[1], 1ull);
                if (flags & REC_HOPS_LIMIT) atomicAdd((unsigned long long *)&R->rstat[2], 1ull);
                atomicAdd((unsigned long long *)&R->rstat[3], (unsigned long long)fo.swept);
                atomicAdd((unsigned long long *)&R->rstat[4], (unsigned long long)fo.arcs);
            }
            if (flags & REC_ARCS_LIMIT) {
                atomicAdd((unsigned long long *)&a.stats[5], 1ull);
                int pos = atomicAdd(&a.retry[0], 1);
                a.retry[1 + pos] = (int32_t)P.q;
            }
        }
        __syncthreads();
    }
    KArgs &a = launch_args();
    if (l == 0) {
        u32 *hdr = a.sl.hdr + slab * 4;
        hdr[0] = serial;
        // load balance of the persistent grid: busy time of this slab, the
        // last finish and the first start (constant-rate wall clock)
        const u64 t_end = wall_clock64();
        atomicAdd((unsigned long long *)&a.stats[9], (unsigned long long)(t_end - t_begin));
        atomicMax((unsigned long long *)&a.stats[10], (unsigned long long)t_end);
        atomicMax((unsigned long long *)&a.stats[11], (unsigned long long)~t_begin);
        // the slab's pair serial, for the host's wrap guard
        atomicMax((unsigned long long *)&a.stats[12], (unsigned long long)serial);
        atomicAdd((unsigned long long *)&a.stats[16], (unsigned long long)fwd_ticks);
        atomicAdd((unsigned long long *)&a.stats[17], (unsigned long long)rev_ticks);
    }
}

// ------------------------------------------------------------ multiword path
// Pairs whose 64-bit counts saturate are taken again with counts of kWide
// limbs (the paper counts with 128-bit and arbitrary-precision integers where
// 64 bits do not suffice).  It is an exactness path, not a fast one: one
// lane per pair runs the forward tick by tick (all reads of a tick before its
// commits; one head run at a time) and the reverse arc by arc, with the same
// commits, arcs, terminal rule and level resets as the batched kernels.
// f = N / sigma is the IEEE quotient of the two counts rounded to double.

struct Wd { u64 w[kWide]; };

__device__ __forceinline__ void wd_set(Wd &a, u64 x) {
    a.w[0] = x;
    for (int i = 1; i < kWide; ++i) a.w[i] = 0;
}
__device__ __forceinline__ void wd_load(Wd &a, const u64 *p) { for (int i = 0; i < kWide; ++i) a.w[i] = p[i]; }
__device__ __forceinline__ void wd_store(u64 *p, const Wd &a) { for (int i = 0; i < kWide; ++i) p[i] = a.w[i]; }
__device__ __forceinline__ bool wd_zero(const Wd &a) {
    u64 x = 0;
    for (int i = 0; i < kWide; ++i) x |= a.w[i];
    return x == 0;
}
__device__ __forceinline__ bool wd_sat(const Wd &a) {
    u64 x = kUMax;
    for (int i = 0; i < kWide; ++i) x &= a.w[i];
    return x == kUMax;
}
__device__ __forceinline__ bool wd_eq(const Wd &a, const Wd &b) {
    u64 x = 0;
    for (int i = 0; i < kWide; ++i) x |= a.w[i] ^ b.w[i];
    return x == 0;
}
__device__ __forceinline__ void wd_fill(Wd &a) { for (int i = 0; i < kWide; ++i) a.w[i] = kUMax; }
// a += b, saturating at 2^(64 kWide) - 1
__device__ __forceinline__ void wd_add(Wd &a, const Wd &b) {
    if (wd_sat(a) || wd_sat(b)) { wd_fill(a); return; }
    u64 carry = 0;
    for (int i = 0; i < kWide; ++i) {
        const u64 x = a.w[i] + b.w[i];
        const u64 c1 = x < a.w[i];
        const u64 y = x + carry;
        const u64 c2 = y < x;
        a.w[i] = y;
        carry = c1 | c2;
    }
    if (carry) wd_fill(a);
}
// a * b, saturating
__device__ __forceinline__ Wd wd_mul(const Wd &a, const Wd &b) {
    Wd r;
    if (wd_sat(a) || wd_sat(b)) { wd_fill(r); return r; }
    u64 acc[2 * kWide];
    for (int i = 0; i < 2 * kWide; ++i) acc[i] = 0;
    for (int i = 0; i < kWide; ++i) {
        u64 carry = 0;
        for (int j = 0; j < kWide; ++j) {
            const u64 lo = a.w[i] * b.w[j], hi = __umul64hi(a.w[i], b.w[j]);
            u64 x = acc[i + j] + lo;
            u64 c = x < lo;
            const u64 y = x + carry;
            c += y < x;
            acc[i + j] = y;
            carry = hi + c;  // no wrap: hi <= 2^64 - 2
        }
        acc[i + kWide] = carry;
    }
    bool over = false;
    for (int i = kWide; i < 2 * kWide; ++i) over |= acc[i] != 0;
    if (over) { wd_fill(r); return r; }
    for (int i = 0; i < kWide; ++i) r.w[i] = acc[i];
    return r;
}
// the count rounded to double, to nearest with ties to even: the top 64 bits
// with a sticky bit for what lies below (the 11 bits under the 53-bit
// significand make the hardware rounding of the 64-bit value exact)
__device__ double wd_to_double(const Wd &a) {
    int i = kWide - 1;
    while (i > 0 && a.w[i] == 0) --i;
    if (i == 0) return (double)a.w[0];
    const u64 hi = a.w[i], lo = a.w[i - 1];
    const int sh = __clzll((long long)hi);
    u64 top = sh ? ((hi << sh) | (lo >> (64 - sh))) : hi;
    bool sticky = sh ? (lo << sh) != 0 : lo != 0;
    for (int j = i - 2; j >= 0; --j) sticky |= a.w[j] != 0;
    if (sticky) top |= 1ull;
    return ldexp((double)top, 64 * i - sh);
}

// the commit of a head run (the rules of head_commit, multiword)
__device__ bool wd_commit(int opt, bool rv, u32 hv, const Wd &Sv, u32 d, const Wd &c, u32 &nh, Wd &nS) {
    if (opt == OPT_SH || opt == OPT_SFM) {
        const u32 hcur = rv ? hv : kHInf;
        if (d > hcur) return false;
        if (d < hcur) { nh = d; nS = c; }
        else { nh = hcur; nS = Sv; wd_add(nS, c); }
        return true;
    }
    if (opt == OPT_FM) {
        const u32 hcur = rv ? hv : kHInf;
        nh = d < hcur ? d : hcur;
        if (rv) nS = Sv; else wd_set(nS, 0);
        wd_add(nS, c);
        return true;
    }
    if (rv) return false;  // pfm: only the earliest arrival counts
    nh = d;
    nS = c;
    return true;
}

__device__ int64_t lb32(const int32_t *arr, int64_t lo, int64_t hi, int32_t x) {  // first >= x
    while (lo < hi) { const int64_t md = (lo + hi) >> 1; if (arr[md] < x) lo = md + 1; else hi = md; }
    return lo;
}

__global__ void __launch_bounds__(64) k_wide(LaunchArgs a_arg, WideSlabs ws) {
    (void)a_arg;
    KArgs &a = launch_args();
    if (threadIdx.x != 0) return;  // one lane per pair: no barriers below
    const int64_t slab = blockIdx.x;
    u64 *ST = ws.ST + slab * ws.nmax, *SS = ws.SS + slab * ws.nmax * kWide;
    u64 *RT = ws.RT + slab * ws.nmax, *RA = ws.RA + slab * ws.nmax * kWide;
    u64 *NV = ws.NV + slab * ws.nmax * kWide;
    int32_t *touched = ws.touched + slab * ws.nmax;
    u32 *TL = ws.TL + slab * ws.gmax;
    u64 *TC = ws.TC + slab * ws.gmax * kWide;
    u64 *AR = ws.AR + slab * ws.cap * (3 + kWide);
    u32 serial = ws.hdr[slab * 4];
    const int64_t np = a.npairs;
    for (;;) {
        const int64_t q = (int64_t)atomicAdd(a.work, 1u);
        if (q >= np) break;
        Pair P;
        resolve_pair<false>(a, q, P);
        serial += 2;
        if (serial < 2u) serial = 2u;
        const u32 ftag = serial, rtag = serial + 1u;
        const int32_t *U = a.g.U, *V = a.g.V, *T = a.g.T;
        // window: first departure of s, last arrival at z, inside [t0, t1]
        const int32_t gs = P.noff + P.s, gz = P.noff + P.z;
        const int64_t o0 = a.g.out_off[gs], o1 = a.g.out_off[gs + 1];
        const int64_t i0 = a.g.in_off[gz], i1 = a.g.in_off[gz + 1];
        const int64_t od = lb32(a.g.out_t, o0, o1, P.t0);
        const int64_t id = (P.t1 == INT32_MAX ? i1 : lb32(a.g.in_t, i0, i1, P.t1 + 1)) - 1;
        u32 flags = 0, zh = kHInf;
        Wd zS;
        wd_set(zS, 0);
        int32_t t_arr = -1;
        int64_t narcs = 0, swept = 0;
        bool ok = od < o1 && id >= i0;
        const int32_t dep = ok ? a.g.out_t[od] : 0, lin = ok ? a.g.in_t[id] : 0;
        ok = ok && dep <= P.t1 && lin >= P.t0 && lin >= dep;
        if (ok) {
            const int64_t lo = lb32(T, P.elo, P.ehi, dep);
            const int64_t hi = lb32(T, lo, P.ehi, lin == INT32_MAX ? lin : lin + 1);
            ST[P.s] = (u64)ftag;  // the origin: 0 hops, one walk
            Wd one;
            wd_set(one, 1);
            wd_store(SS + (int64_t)P.s * kWide, one);
            bool done = false;
            for (int64_t i = lo; i < hi && !done && !flags;) {
                const int32_t t = T[i];
                int64_t j = i + 1;
                while (j < hi && T[j] == t) ++j;
                // reads: every tail's state before the tick
                for (int64_t e = i; e < j; ++e) {
                    const int32_t u = U[e];
                    const u64 st = ST[u];
                    if ((u32)st == ftag) {
                        TL[e - i] = (u32)(st >> 32) & 0xFFFFu;
                        Wd x;
                        wd_load(x, SS + (int64_t)u * kWide);
                        wd_store(TC + (e - i) * kWide, x);
                    } else {
                        TL[e - i] = kHInf;
                    }
                }
                bool zhit = false;
                // one head run at a time (the tick's edges are sorted by head)
                for (int64_t r0 = i, r1; r0 < j; r0 = r1) {
                    const int32_t v = V[r0];
                    r1 = r0 + 1;
                    while (r1 < j && V[r1] == v) ++r1;
                    u32 d = 0xFFFFFFFFu;
                    for (int64_t e = r0; e < r1; ++e)
                        if (TL[e - i] != kHInf && TL[e - i] + 1 < d) d = TL[e - i] + 1;
                    if (d == 0xFFFFFFFFu) continue;  // no reached tail
                    if (d >= kHInf) { flags |= REC_HOPS_LIMIT; break; }
                    Wd c;
                    wd_set(c, 0);
                    for (int64_t e = r0; e < r1; ++e) {
                        const u32 h = TL[e - i];
                        if (h == kHInf || (P.level && h + 1 != d)) continue;
                        Wd x;
                        wd_load(x, TC + (e - i) * kWide);
                        wd_add(c, x);
                    }
                    const u64 sv = ST[v];
                    const bool rv = (u32)sv == ftag;
                    Wd Sv, nS;
                    if (rv) wd_load(Sv, SS + (int64_t)v * kWide); else wd_set(Sv, 0);
                    u32 nh = 0;
                    if (!wd_commit(P.opt, rv, rv ? (u32)(sv >> 32) & 0xFFFFu : 0u, Sv, d, c, nh, nS)) continue;
                    ST[v] = (u64)ftag | ((u64)nh << 32);
                    wd_store(SS + (int64_t)v * kWide, nS);
                    // arcs of the run's counted tails
                    for (int64_t e = r0; e < r1; ++e) {
                        const u32 h = TL[e - i];
                        if (h == kHInf || (P.level && h + 1 != d)) continue;
                        if (narcs >= ws.cap) { flags |= REC_ARCS_LIMIT; break; }
                        u64 *ar = AR + narcs * (3 + kWide);
                        ar[0] = (u64)(u32)v | ((u64)(u32)t << 32);
                        ar[1] = (u64)(u32)e | ((u64)(u32)U[e] << 32);
                        ar[2] = (u64)h | ((u64)d << 16);
                        for (int w = 0; w < kWide; ++w) ar[3 + w] = TC[(e - i) * kWide + w];
                        ++narcs;
                    }
                    if (v == P.z) {
                        if (P.opt == OPT_SH) { if (nh < zh) t_arr = t; }
                        else t_arr = t;
                        zh = nh;
                        zS = nS;
                        zhit = true;
                    }
                }
                swept = j - lo;
                if (zhit && P.opt != OPT_SH) done = true;
                i = j;
            }
        }
        // reverse over the arcs, newest first, a tick at a time
        const bool reach = ok && zh != kHInf && !(flags & (REC_HOPS_LIMIT | REC_ARCS_LIMIT));
        bool sat = reach && wd_sat(zS);
        int64_t ntouch = 0;
        if (reach && !sat) {
            const double sg = wd_to_double(zS);
            for (int64_t ac = narcs; ac > 0;) {
                const int32_t t = (int32_t)(AR[(ac - 1) * (3 + kWide)] >> 32);
                int64_t a0 = ac - 1;
                while (a0 > 0 && (int32_t)(AR[(a0 - 1) * (3 + kWide)] >> 32) == t) --a0;
                // heads: B(head appearance) from state older than the tick
                for (int64_t x = a0; x < ac; ++x) {
                    const u64 *ar = AR + x * (3 + kWide);
                    const int32_t v = (int32_t)(u32)ar[0];
                    const u32 hl = (u32)(ar[2] >> 16) & 0xFFFFu;
                    Wd B;
                    if (v == P.z) wd_set(B, (P.opt != OPT_SH || hl == zh) ? 1ull : 0ull);
                    else {
                        const u64 rt = RT[v];
                        if ((u32)rt == rtag && (!P.level || ((u32)(rt >> 32) & 0xFFFFu) == hl))
                            wd_load(B, RA + (int64_t)v * kWide);
                        else wd_set(B, 0);
                    }
                    wd_store(TC + (x - a0) * kWide, B);
                }
                // N(e) = tail count * B(head), N(v) of the head, f(e)
                for (int64_t x = a0; x < ac; ++x) {
                    const u64 *ar = AR + x * (3 + kWide);
                    Wd B, tc;
                    wd_load(B, TC + (x - a0) * kWide);
                    if (wd_zero(B)) continue;
                    wd_load(tc, ar + 3);
                    const Wd na = wd_mul(tc, B);
                    if (wd_sat(na)) sat = true;
                    const int32_t v = (int32_t)(u32)ar[0];
                    const u32 k = (u32)ar[1];
                    if (v != P.s && v != P.z) {
                        Wd nv;
                        wd_load(nv, NV + (int64_t)v * kWide);
                        if (wd_zero(nv)) touched[ntouch++] = v;
                        wd_add(nv, na);
                        if (wd_sat(nv)) sat = true;
                        wd_store(NV + (int64_t)v * kWide, nv);
                    }
                    const double fe = wd_to_double(na) / sg;
                    if (P.req->Esum) atomicAdd(&P.req->Esum[k], fe);
                    if (a.edge_f) a.edge_f[P.qout * a.g.m + k] = fe;
                }
                // tails: level resets, then the additions
                for (int64_t x = a0; x < ac; ++x) {
                    const u64 *ar = AR + x * (3 + kWide);
                    Wd B;
                    wd_load(B, TC + (x - a0) * kWide);
                    if (wd_zero(B)) continue;
                    const int32_t u = (int32_t)(ar[1] >> 32);
                    const u32 want = P.level ? (u32)ar[2] & 0xFFFFu : 0u;
                    const u64 rt = RT[u];
                    if ((u32)rt != rtag || ((u32)(rt >> 32) & 0xFFFFu) != want) {
                        RT[u] = (u64)rtag | ((u64)want << 32);
                        Wd zero;
                        wd_set(zero, 0);
                        wd_store(RA + (int64_t)u * kWide, zero);
                    }
                }
                for (int64_t x = a0; x < ac; ++x) {
                    const u64 *ar = AR + x * (3 + kWide);
                    Wd B, acc;
                    wd_load(B, TC + (x - a0) * kWide);
                    if (wd_zero(B)) continue;
                    const int32_t u = (int32_t)(ar[1] >> 32);
                    wd_load(acc, RA + (int64_t)u * kWide);
                    wd_add(acc, B);
                    wd_store(RA + (int64_t)u * kWide, acc);
                }
                ac = a0;
            }
            // flow conservation at the origin: B(origin) = sigma
            Wd bo;
            const u64 rt = RT[P.s];
            if ((u32)rt == rtag && (!P.level || ((u32)(rt >> 32) & 0xFFFFu) == 0u)) wd_load(bo, RA + (int64_t)P.s * kWide);
            else wd_set(bo, 0);
            if (!sat && !wd_eq(bo, zS)) flags |= REC_SELFCHECK;
            if (sat && a.edge_f)
                for (int64_t x = 0; x < narcs; ++x) a.edge_f[P.qout * a.g.m + (u32)AR[x * (3 + kWide) + 1]] = 0.0;
            // finalize: f(v) = N(v) / sigma into the sums; N back to zero
            const DevReq *R = P.req;
            for (int64_t x = 0; x < ntouch; ++x) {
                const int32_t v = touched[x];
                Wd nv;
                wd_load(nv, NV + (int64_t)v * kWide);
                Wd zero;
                wd_set(zero, 0);
                wd_store(NV + (int64_t)v * kWide, zero);
                if (sat) continue;
                const double f = wd_to_double(nv) / sg;
                const int64_t gv = (int64_t)P.noff + v;
                if (R->Bsum) atomicAdd(&R->Bsum[gv], f);
                if (R->Wsum) atomicAdd(&R->Wsum[gv], f * f);
                if (R->Rsum)
                    for (int jc = 0; jc < P.c; ++jc)
                        atomicAdd(&R->Rsum[gv * P.c + jc], ((P.lam >> jc) & 1ull) ? -f : f);
                if (a.node_f) a.node_f[P.qout * (int64_t)a.g.n_total + gv] = f;
            }
        }
        bool big = false;  // sigma beyond 64 bits
        for (int w = 1; w < kWide; ++w) big |= zS.w[w] != 0;
        if (sat) flags |= REC_OVERFLOW;
        if (reach && big) flags |= REC_WIDE;
        if (a.rec) {
            int32_t *rr = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(a.rec) + P.qout * 24);
            rr[0] = reach ? 1 : 0;
            rr[1] = reach ? t_arr : -1;
            rr[2] = reach ? (int32_t)zh : -1;
            rr[3] = (int32_t)flags;
            *reinterpret_cast<u64 *>(rr + 4) = reach ? (big ? kUMax : zS.w[0]) : 0ull;
        }
        const DevReq *R = P.req;
        if (flags & REC_OVERFLOW) atomicAdd((unsigned long long *)&a.stats[2], 1ull);
        if (flags & REC_SELFCHECK) atomicAdd((unsigned long long *)&a.stats[6], 1ull);
        if (flags & (REC_ARCS_LIMIT | REC_HOPS_LIMIT)) atomicAdd((unsigned long long *)&a.stats[4], 1ull);
        if (R->rstat) {
            if (flags & REC_OVERFLOW) atomicAdd((unsigned long long *)&R->rstat[0], 1ull);
            if (flags & (REC_HOPS_LIMIT | REC_ARCS_LIMIT)) atomicAdd((unsigned long long *)&R->rstat[2], 1ull);
        }
        (void)swept;
    }
    ws.hdr[slab * 4] = serial;
    atomicMax((unsigned long long *)&a.stats[12], (unsigned long long)serial);
}

// ------------------------------------------------------------ pair order

// first index in [a, b) with arr[i] >= x (arr ascending), one thread
__device__ int64_t lower_bound_1(const int32_t *arr, int64_t a, int64_t b, int32_t x) {
    while (a < b) {
        const int64_t m = a + (b - a) / 2;
        if (arr[m] < x) a = m + 1; else b = m;
    }
    return a;
}

// Cost estimate of every launch slot's pair, in edges of the time-sorted
// stream: the window from the first departure of s to the last arrival at z
// (exact for sh, which sweeps all of it); for the optimalities that stop at
// the first arrival at z, the window up to z's kPairKeyK-th in-edge after the
// departure (z's arrival cannot come earlier than its first in-edge, and
// targets with few in-edges are the ones reached late).  The launch runs the
// slots in decreasing order of the estimate, bucketed on a log scale with
// four buckets per octave (a counting sort: histogram, scan, scatter), so
// that the longest sweeps start first.
constexpr int kPairKeyK = 8;

__device__ __forceinline__ u32 order_bucket(u64 est) {
    const u64 x = est + 1;
    const int e = 63 - __clzll((long long)x);
    const u32 frac = e >= 2 ? (u32)((x >> (e - 2)) & 3ull) : (u32)((x << (2 - e)) & 3ull);
    const u32 b = 4u * (u32)e + frac;
    return b < (u32)kOrderBuckets ? b : (u32)kOrderBuckets - 1;
}

__global__ void __launch_bounds__(256) k_pair_keys(LaunchArgs a, u32 *bucket, u64 *hist) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= (a.npairs_dev ? *a.npairs_dev : a.npairs)) return;
    a.pq = nullptr;
    Pair P;
    resolve_pair(a, slot, P);
    if (P.req->mode == MODE_DISTANCES || P.req->mode == MODE_RTB) { P.single = true; P.z = -1; }
    const int32_t gs = P.noff + P.s;
    const int64_t o0 = a.g.out_off[gs], o1 = a.g.out_off[gs + 1];
    const int64_t od = lower_bound_1(a.g.out_t, o0, o1, P.t0);
    u64 est = 0;
    if (P.single) {
        // a single source: from its first departure to the window's end
        if (od < o1 && a.g.out_t[od] <= P.t1) {
            const int64_t lo = lower_bound_1(a.g.T, P.elo, P.ehi, a.g.out_t[od]);
            const int64_t hi = lower_bound_1(a.g.T, lo, P.ehi, P.t1 == INT32_MAX ? P.t1 : P.t1 + 1);
            est = (u64)(hi - lo);
        }
        const u32 b = order_bucket(est);
        bucket[slot] = b;
        atomicAdd((unsigned long long *)&hist[b], 1ull);
        return;
    }
    const int32_t gz = P.noff + P.z;
    const int64_t i0 = a.g.in_off[gz], i1 = a.g.in_off[gz + 1];
    const int64_t id = lower_bound_1(a.g.in_t, i0, i1, P.t1 == INT32_MAX ? P.t1 : P.t1 + 1) - 1;
    if (od < o1 && id >= i0) {
        const int32_t dep = a.g.out_t[od], lin = a.g.in_t[id];
        if (dep <= P.t1 && lin >= P.t0 && lin >= dep) {
            int32_t tend = lin;
            if (P.opt != OPT_SH) {
                const int64_t j = lower_bound_1(a.g.in_t, i0, id + 1, dep == INT32_MAX ? dep : dep + 1) + (kPairKeyK - 1);
                tend = a.g.in_t[j < id ? j : id];
            }
            const int64_t lo = lower_bound_1(a.g.T, P.elo, P.ehi, dep);
            const int64_t hi = lower_bound_1(a.g.T, lo, P.ehi, tend == INT32_MAX ? tend : tend + 1);
            est = (u64)(hi - lo);
        }
    }
    const u32 b = order_bucket(est);
    bucket[slot] = b;
    atomicAdd((unsigned long long *)&hist[b], 1ull);
}

// cursor[b] = number of slots in buckets above b (one thread: kOrderBuckets steps)
__global__ void k_order_scan(u64 *hist) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    u64 run = 0;
    for (int b = kOrderBuckets - 1; b >= 0; --b) {
        const u64 h = hist[b];
        hist[b] = run;
        run += h;
    }
}

__global__ void __launch_bounds__(256) k_order_scatter(int64_t npairs, const int64_t *npairs_dev, const u32 *bucket,
                                                       u64 *cursor, int32_t *order) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= (npairs_dev ? *npairs_dev : npairs)) return;
    const u64 pos = atomicAdd((unsigned long long *)&cursor[bucket[slot]], 1ull);
    order[pos] = (int32_t)slot;
}

// ------------------------------------------------------------ reductions

// per block: max_v W[v], sum_v B[v], max_v R[v][j] (j < c)
__global__ void __launch_bounds__(256) k_reduce(ReduceArgs a) {
    __shared__ double sh[256];
    const int tid = threadIdx.x;
    const int64_t nb = gridDim.x;
    const int64_t per = (a.n + nb - 1) / nb;
    const int64_t v0 = blockIdx.x * per;
    const int64_t v1 = (v0 + per < a.n) ? v0 + per : a.n;
    double* out = a.part + blockIdx.x * (int64_t)(2 + a.c);
    // W max
    double x = -1.0 / 0.0;
    for (int64_t v = v0 + tid; v < v1; v += 256) x = fmax(x, a.W[v]);
    sh[tid] = x;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) { if (tid < s) sh[tid] = fmax(sh[tid], sh[tid + s]); __syncthreads(); }
    if (tid == 0) out[0] = sh[0];
    __syncthreads();
    // B sum (fixed order: strided partials, then a tree)
    x = 0.0;
    for (int64_t v = v0 + tid; v < v1; v += 256) x += a.B[v];
    sh[tid] = x;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) { if (tid < s) sh[tid] = sh[tid] + sh[tid + s]; __syncthreads(); }
    if (tid == 0) out[1] = sh[0];
    __syncthreads();
    for (int j = 0; j < a.c; ++j) {
        x = -1.0 / 0.0;
        for (int64_t v = v0 + tid; v < v1; v += 256) x = fmax(x, a.R[v * a.c + j]);
        sh[tid] = x;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) { if (tid < s) sh[tid] = fmax(sh[tid], sh[tid + s]); __syncthreads(); }
        if (tid == 0) out[2 + j] = sh[0];
        __syncthreads();
    }
}

__global__ void k_zero_u32(u32 *a, u32 *b, u32 *c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) { *a = 0u; *b = 0u; if (c) *c = 0u; }
}

__global__ void k_fill_u64(u64 *p, u64 val, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = val;
}

}  // namespace mantra

// ------------------------------------------------------------ launchers

extern "C" {
// the multiword path over the pairs a->pq names (one lane per pair)
hipError_t mantra_launch_wide(const mantra::LaunchArgs *a, const mantra::WideSlabs *ws, int nslabs, hipStream_t st) {
    hipLaunchKernelGGL(mantra::k_wide, dim3(nslabs), dim3(64), 0, st, *a, *ws);
    return hipGetLastError();
}
hipError_t mantra_launch_sweep(const mantra::LaunchArgs *a, int nslabs, size_t lds_bytes, hipStream_t st) {
    if (a->lds_bitmap)
        hipLaunchKernelGGL((mantra::k_sweep<mantra::MODE_PAIRS, false>), dim3(nslabs), dim3(64), lds_bytes, st, *a);
    else
        hipLaunchKernelGGL((mantra::k_sweep<mantra::MODE_PAIRS, true>), dim3(nslabs), dim3(64), lds_bytes, st, *a);
    return hipGetLastError();
}
// the single-source (distance) form of the sweep
hipError_t mantra_launch_sweep_sources(const mantra::LaunchArgs *a, int nslabs, size_t lds_bytes, hipStream_t st) {
    if (a->lds_bitmap)
        hipLaunchKernelGGL((mantra::k_sweep<mantra::MODE_DISTANCES, false>), dim3(nslabs), dim3(64), lds_bytes, st, *a);
    else
        hipLaunchKernelGGL((mantra::k_sweep<mantra::MODE_DISTANCES, true>), dim3(nslabs), dim3(64), lds_bytes, st, *a);
    return hipGetLastError();
}
// the sweep with the RTB estimator (sources, all targets; needs the slabs' T)
hipError_t mantra_launch_sweep_rtb(const mantra::LaunchArgs *a, int nslabs, size_t lds_bytes, hipStream_t st) {
    if (a->lds_bitmap)
        hipLaunchKernelGGL((mantra::k_sweep<mantra::MODE_RTB, false>), dim3(nslabs), dim3(64), lds_bytes, st, *a);
    else
        hipLaunchKernelGGL((mantra::k_sweep<mantra::MODE_RTB, true>), dim3(nslabs), dim3(64), lds_bytes, st, *a);
    return hipGetLastError();
}
// the sweep with the TRK estimator (one sampled optimal walk per pair)
hipError_t mantra_launch_sweep_trk(const mantra::LaunchArgs *a, int nslabs, size_t lds_bytes, hipStream_t st) {
    if (a->lds_bitmap)
        hipLaunchKernelGGL((mantra::k_sweep<mantra::MODE_TRK, false>), dim3(nslabs), dim3(64), lds_bytes, st, *a);
    else
        hipLaunchKernelGGL((mantra::k_sweep<mantra::MODE_TRK, true>), dim3(nslabs), dim3(64), lds_bytes, st, *a);
    return hipGetLastError();
}
hipError_t mantra_launch_reduce(const mantra::ReduceArgs *a, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(mantra::k_reduce, dim3(blocks), dim3(256), 0, st, *a);
    return hipGetLastError();
}
hipError_t mantra_launch_fill(mantra::u64 *p, mantra::u64 val, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(mantra::k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, st, p, val, n);
    return hipGetLastError();
}
// slot order of a launch, longest estimated sweep first: order[npairs];
// bucket[npairs] and hist[kOrderBuckets] are scratch
hipError_t mantra_launch_order(const mantra::LaunchArgs *a, mantra::u32 *bucket, mantra::u64 *hist,
                               int32_t *order, hipStream_t st) {
    if (a->npairs <= 0) return hipSuccess;
    const int64_t blocks = (a->npairs + 255) / 256;
    hipLaunchKernelGGL(mantra::k_fill_u64, dim3(1), dim3(256), 0, st, hist, 0ull, (int64_t)mantra::kOrderBuckets);
    hipLaunchKernelGGL(mantra::k_pair_keys, dim3((unsigned)blocks), dim3(256), 0, st, *a, bucket, hist);
    hipLaunchKernelGGL(mantra::k_order_scan, dim3(1), dim3(64), 0, st, hist);
    hipLaunchKernelGGL(mantra::k_order_scatter, dim3((unsigned)blocks), dim3(256), 0, st, a->npairs, a->npairs_dev,
                       (const mantra::u32 *)bucket, hist, order);
    return hipGetLastError();
}
// zero the launch counters (work counter, retry and multiword counts (may be
// null), statistics) with kernels, so that the sequence can be captured in a
// graph
hipError_t mantra_launch_clear(mantra::u32 *work, mantra::u32 *retry, mantra::u32 *wide, mantra::u64 *stats,
                               hipStream_t st) {
    hipLaunchKernelGGL(mantra::k_zero_u32, dim3(1), dim3(64), 0, st, work, retry, wide);
    hipLaunchKernelGGL(mantra::k_fill_u64, dim3(1), dim3(64), 0, st, stats, 0ull, (int64_t)mantra::kStats);
    return hipGetLastError();
}
// LDS of a sweep workgroup ahead of its bitmap and hub state: the tables of
// the forward and reverse sweeps, and the chunk table's first entries
size_t mantra_tab_lds_bytes(void) { return sizeof(mantra::TabLds) + sizeof(mantra::u32) * mantra::kXtLds; }
// resident sweep workgroups per CU for a given dynamic LDS size (gbm: the
// instance with the reached set in global memory)
int mantra_sweep_occupancy(size_t lds_bytes, int gbm) {
    int nb = 0;
    const hipError_t e =
        gbm ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mantra::k_sweep<mantra::MODE_PAIRS, true>, 64, lds_bytes)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mantra::k_sweep<mantra::MODE_PAIRS, false>, 64, lds_bytes);
    return e == hipSuccess ? nb : 0;
}
}
