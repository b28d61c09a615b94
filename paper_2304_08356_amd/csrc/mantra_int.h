// Library-internal declarations shared by the host runtime and the serving
// scheduler (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <stdio.h>
#include <stdarg.h>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mantra_dev.h"
#include "../../include/mantra.h"

extern "C" {
hipError_t mantra_launch_sweep(const mantra::LaunchArgs *a, int nslabs, size_t lds_bytes, hipStream_t st);
hipError_t mantra_launch_sweep_sources(const mantra::LaunchArgs *a, int nslabs, size_t lds_bytes, hipStream_t st);
hipError_t mantra_launch_sweep_trk(const mantra::LaunchArgs *a, int nslabs, size_t lds_bytes, hipStream_t st);
hipError_t mantra_launch_sweep_rtb(const mantra::LaunchArgs *a, int nslabs, size_t lds_bytes, hipStream_t st);
hipError_t mantra_launch_reduce(const mantra::ReduceArgs *a, int blocks, hipStream_t st);
hipError_t mantra_launch_fill(mantra::u64 *p, mantra::u64 val, int64_t n, hipStream_t st);
hipError_t mantra_launch_clear(mantra::u32 *work, mantra::u32 *retry, mantra::u32 *wide, mantra::u64 *stats,
                               hipStream_t st);
hipError_t mantra_launch_wide(const mantra::LaunchArgs *a, const mantra::WideSlabs *ws, int nslabs, hipStream_t st);
hipError_t mantra_launch_order(const mantra::LaunchArgs *a, mantra::u32 *bucket, mantra::u64 *hist,
                               int32_t *order, hipStream_t st);
size_t mantra_tab_lds_bytes(void);
int mantra_sweep_occupancy(size_t lds_bytes, int gbm);
}

namespace mantra {

// ------------------------------------------------------------------ errors

extern thread_local std::string g_err;
// sets the thread's error text and returns code
int fail(int code, const char *fmt, ...);

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            if (e_ == hipErrorOutOfMemory) return fail(MANTRA_E_OOM, "%s: %s", #expr,     \
                                                       hipGetErrorString(e_));            \
            return fail(MANTRA_E_INTERNAL, "%s: %s", #expr, hipGetErrorString(e_));       \
        }                                                                                 \
    } while (0)

// outputs pass to the host in pieces of this many values
constexpr int64_t kOutChunk = (int64_t)1 << 22;

template <class T>
static inline hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, sizeof(T) * (count ? count : 1));
}

// ------------------------------------------------------------------ graph

struct SlabPool {
    int nslabs = 0;
    int64_t nmax = 0, cap = 0, gmax = 0;
    u64 *F = nullptr, *N = nullptr, *AG = nullptr, *arcs = nullptr, *XS = nullptr;
    u64 *T = nullptr;  // RTB launches only: first arrivals, [nslabs][nmax][2]
    unsigned char *BM = nullptr;  // reached-set bitmaps (graphs whose bitmap is not in LDS)
    u32 *hdr = nullptr;
    int32_t *touched = nullptr;
    // shared arc chunks for pairs whose arcs pass the slab's own buffer
    u64 *xarcs = nullptr;
    u32 *xfree = nullptr, *xtab = nullptr;
    int64_t nchunks = 0, xmax = 0;
    // largest pair serial of any slab (the wrap guard)
    u64 serial_hi = 0;
    void release() {
        hipFree(F); hipFree(N); hipFree(AG); hipFree(arcs); hipFree(XS); hipFree(T); hipFree(BM);
        hipFree(hdr); hipFree(touched); hipFree(xarcs); hipFree(xfree); hipFree(xtab);
        F = N = AG = arcs = XS = T = xarcs = nullptr;
        BM = nullptr;
        hdr = xfree = xtab = nullptr;
        touched = nullptr;
        nslabs = 0;
        nchunks = xmax = 0;
        serial_hi = 0;
    }
    DevSlabs view() const {
        DevSlabs s;
        s.F = F; s.N = N; s.T = T; s.AG = AG; s.touched = touched; s.arcs = arcs;
        s.XS = XS; s.BM = BM; s.hdr = hdr; s.nmax = nmax; s.cap = cap; s.gmax = gmax;
        s.xarcs = xarcs; s.xfree = xfree; s.xtab = xtab; s.xwords = (nchunks + 31) / 32; s.xmax = xmax;
        return s;
    }
};

// per-slab state of the multiword path, allocated on its first use
struct WidePool {
    int nslabs = 0;
    int64_t nmax = 0, cap = 0, gmax = 0;
    u64 *ST = nullptr, *SS = nullptr, *RT = nullptr, *RA = nullptr, *NV = nullptr, *TC = nullptr, *AR = nullptr;
    u32 *TL = nullptr, *hdr = nullptr;
    int32_t *touched = nullptr;
    u64 serial_hi = 0;  // largest pair serial of any slab (the wrap guard)
    void release() {
        hipFree(ST); hipFree(SS); hipFree(RT); hipFree(RA); hipFree(NV); hipFree(TC); hipFree(AR);
        hipFree(TL); hipFree(hdr); hipFree(touched);
        ST = SS = RT = RA = NV = TC = AR = nullptr;
        TL = hdr = nullptr;
        touched = nullptr;
        nslabs = 0;
        serial_hi = 0;
    }
    WideSlabs view() const {
        WideSlabs w;
        w.ST = ST; w.SS = SS; w.RT = RT; w.RA = RA; w.NV = NV; w.touched = touched; w.TL = TL; w.TC = TC;
        w.AR = AR; w.hdr = hdr; w.nmax = nmax; w.cap = cap; w.gmax = gmax;
        return w;
    }
};

struct ServeState;  // mantra_serve.hip

}  // namespace mantra

// the opaque handle of the C ABI
struct mantra_graph {
    int device = 0;
    int32_t n_total = 0, G = 1, nmax = 0;
    int64_t m_in = 0, m = 0, ndup = 0, gmax = 1;
    int32_t tmin = 0, tmax = 0;
    std::vector<int32_t> seg_noff;
    std::vector<int64_t> seg_eoff;
    std::vector<int64_t> in2k;  // input edge index -> internal edge id
    std::vector<int32_t> perm;  // input node id (global) -> internal id, hubs first
    std::vector<int32_t> iperm; // internal id -> input id
    int32_t *dU = nullptr, *dV = nullptr, *dT = nullptr, *dout_t = nullptr, *din_t = nullptr,
            *dseg_noff = nullptr, *dperm = nullptr;
    uint32_t *din2k = nullptr;      // [m_in] input edge index -> internal edge id
    double *dout = nullptr;         // [kOutChunk] outputs in the caller's order, on their way to the host
    int64_t *dout_off = nullptr, *din_off = nullptr, *dseg_eoff = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    mantra::SlabPool pool, pool_big;
    mantra::WidePool wide;          // the multiword path's slabs (first use)
    int32_t *dwide = nullptr;       // [1 + slots] pairs for the multiword path
    int64_t wide_cap = 0;
    int user_slabs = 0;
    int64_t user_cap = 0;
    int no_chunks = 0;              // no shared arc chunks (launch option)
    int64_t max_chunks = 0;         // > 0: at most this many shared arc chunks (launch option)
    int order_mode = MANTRA_ORDER_LONGEST_FIRST;
    int hub_nodes = 0;              // forward state of nodes below this id in LDS
    int wide_mode = MANTRA_WIDE_NOT_FM;  // which saturated pairs take the multiword path
    int graph_rounds = 0;
    int per_pair = 0;               // unbatched form: one launch per pair
    int64_t *dnp = nullptr;         // pair count of a graph replay
    // launch order scratch
    mantra::u32 *dbucket = nullptr;
    int32_t *dorder = nullptr;
    mantra::u64 *dhist = nullptr;
    int64_t order_cap = 0;
    // misc device buffers
    mantra::u32 *dwork = nullptr;
    mantra::u64 *dstats = nullptr;
    int32_t *dretry = nullptr;
    int64_t retry_cap = 0;
    double *dpart = nullptr;
    int part_blocks = 0, part_c = -1;
    mantra::DevReq *dreqs = nullptr;
    int dreq_cap = 0;
    std::mutex mu;  // one blocking call at a time per graph
    // timing of the last blocking call
    double last_ms = 0;
    int64_t last_launches = 0, last_W = 0, last_arcs = 0, last_tn = 0, last_te = 0, last_live = 0, last_dead = 0;
    int64_t last_fwd_ticks = 0, last_rev_ticks = 0;
    double last_busy_ms = 0;
    mantra::ServeState *serve = nullptr;
    mantra::DevGraph dev() const {
        mantra::DevGraph d;
        d.U = dU; d.V = dV; d.T = dT; d.out_off = dout_off; d.out_t = dout_t; d.in_off = din_off;
        d.in_t = din_t; d.seg_eoff = dseg_eoff; d.seg_noff = dseg_noff; d.n_total = n_total;
        d.G = G; d.m = m; d.perm = dperm;
        return d;
    }
};

namespace mantra {


// ------------------------------------------------------------------ launches

struct LaunchSpec {
    std::vector<DevReq> reqs;
    int64_t npairs = 0;
    const int32_t *dpg = nullptr, *dps = nullptr, *dpz = nullptr;
    void *drec = nullptr;
    double *dnode_f = nullptr, *dedge_f = nullptr;
    int mode = MODE_PAIRS;  // the kernel: MODE_PAIRS, MODE_TRK (pairs), MODE_DISTANCES or MODE_RTB (sources)
};

// what one call of run_sweep did: launch statistics (indices as in
// LaunchArgs::stats), device time of its launches and their count
struct SweepOut {
    u64 st[kStats];
    double ms = 0;
    double first_ms = 0;   // the persistent launch alone (without re-runs)
    int launches = 0;
    double balance = 1.0;  // busy share of the persistent grid
    bool reduced = false;  // the graph replay also ran the request's reduction
};

// the launch sequence of one request's progressive rounds as a HIP graph
struct RoundGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t cap = 0;                  // launch slots it was captured for
    LaunchArgs args;                  // kernel arguments at capture
    int ns = 0;
    const double *W = nullptr, *B = nullptr, *R = nullptr;  // the reduction's sums
    int c = 0;
    void release();
};

int run_sweep(mantra_graph *g, const LaunchSpec &sp, SweepOut &o, RoundGraph *rg = nullptr);
// the work and device time mantra_last_timing reports: cleared by each
// blocking call, summed over its launches
void timing_reset(mantra_graph *g);
void timing_add(mantra_graph *g, const SweepOut &o);
int reduce_blocks(int64_t n);
int reduce_part_ensure(mantra_graph *g, int c);
// persistent workgroups of a launch on this graph
int auto_slabs(const mantra_graph *g);
// the reached set of a pair: a bitmap in LDS (graphs of up to 65,536 nodes),
// else in the slab's global memory; bytes of that per slab (0 with LDS)
int lds_bitmap_ok(int64_t nmax);
size_t node_bytes_per_slab(int64_t nmax);
// dynamic LDS of a sweep workgroup on this graph (its hub setting included)
size_t lds_bytes(const mantra_graph *g);
// default device bytes of the serving scheduler's per-request sums (the slab
// pool's share of the device reserved)
size_t serve_sums_budget(const mantra_graph *g);

// per-request device accumulators of Section 4.2: sums of f, f^2 and the c
// Rademacher-weighted sums per node; sums of f per temporal edge
struct Acc {
    double *B = nullptr, *W = nullptr, *R = nullptr, *E = nullptr;
    int64_t n = 0, m = 0;
    int c = 0;
    void release() { hipFree(B); hipFree(W); hipFree(R); hipFree(E); B = W = R = E = nullptr; }
};

// per-request device counters filled by the sweep kernel
enum { RS_OVERFLOW = 0, RS_REACHABLE = 1, RS_HOPS = 2, RS_WINDOW = 3, RS_ARCS = 4, RS_N = 8 };

// ------------------------------------------------------------------ requests

// One request as a resumable state machine: phases of pairs (the bootstrap
// sample, then the rounds of the progressive schedule, or one fixed sample),
// each cut into slices that launches may share with other requests.
struct ReqRun {
    mantra_request rq;
    int c = 25;
    bool edges = false;
    mantra_result R;
    Acc acc, boot;
    u64 *rstat = nullptr;          // device [RS_N]
    enum { BOOT = 0, ROUND = 1, DONE = 2 } phase = BOOT;
    int64_t prev = 0;              // first pair index of the current phase in its stream
    int64_t target = 0;            // end of the current phase (exclusive)
    int64_t issued = 0;            // pairs of the phase handed to launches
    int64_t om = 0;
    int round = 0;
    RoundGraph rg;                 // graph of the rounds (blocking calls with graph_rounds)
    bool reduced = false;          // the last launch already ran the phase reduction
    int rc = MANTRA_OK;
    std::string err;               // error text of rc
    std::chrono::steady_clock::time_point t_start;  // submission (set by req_begin if unset)
    size_t mem_bytes = 0;          // device bytes the request holds while active
};

int check_request(const mantra_graph *g, const mantra_request &rq);
// device bytes a request needs for its accumulators (admission unit)
size_t req_mem_bytes(const mantra_graph *g, const mantra_request &rq);
// validate, allocate and enter the first phase
int req_begin(mantra_graph *g, ReqRun &q);
// pairs of the current phase not yet handed to a launch
static inline int64_t req_pending(const ReqRun &q) { return q.phase == ReqRun::DONE ? 0 : q.target - q.prev - q.issued; }
// slice of the next count pairs of the current phase at launch slot qoff
DevReq req_slice(ReqRun &q, int64_t count, int64_t qoff);
// after a launch: when the phase is complete, run its reduction and the
// bound checks and move to the next phase (or DONE)
int req_advance(mantra_graph *g, ReqRun &q);
// outputs to the caller's buffers, release device memory, fill the result
int req_finish(mantra_graph *g, ReqRun &q, mantra_result *out);
void req_release(ReqRun &q);

// stop the graph's serving scheduler, failing what it still holds
void serve_stop(mantra_graph *g);

}  // namespace mantra
