// Host runtime of the temporal-betweenness library: graph residency, the
// per-slab device state, launches of the sweep kernel, the progressive
// sampling driver of Algorithm 1, and the serving scheduler.

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

using namespace mantra;

extern "C" {
hipError_t mantra_launch_sweep(const mantra::LaunchArgs *a, int nslabs, size_t lds_bytes, hipStream_t st);
hipError_t mantra_launch_reduce(const mantra::ReduceArgs *a, int blocks, hipStream_t st);
hipError_t mantra_launch_fill(mantra::u64 *p, mantra::u64 val, int64_t n, hipStream_t st);
size_t mantra_tab_lds_bytes(void);
int mantra_sweep_occupancy(size_t lds_bytes);
}

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            if (e_ == hipErrorOutOfMemory) return fail(MANTRA_E_OOM, "%s: %s", #expr,     \
                                                       hipGetErrorString(e_));            \
            return fail(MANTRA_E_INTERNAL, "%s: %s", #expr, hipGetErrorString(e_));       \
        }                                                                                 \
    } while (0)

template <class T>
static hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, sizeof(T) * (count ? count : 1));
}

// ------------------------------------------------------------------ bounds
// Theorem 1 (Eqs. (1)-(3)), Theorem 3's numeric sample size, Hoeffding's
// union bound (Section 4.2), the bootstrap size s' = ln(1/delta)/eps and the
// first schedule element (least s whose Eq. (3) with R = 0 is <= eps).

namespace bnd {
static double xi(double Rc, double W, double vhat, int c, double r, double delta) {
    const double L = log(4.0 / delta);
    double Rt = Rc + sqrt(4.0 * W * L / ((double)c * r));
    if (Rt < 0.0) Rt = 0.0;
    const double Lr = L / r;
    const double R = Rt + Lr + sqrt(Lr * Lr + 2.0 * L * Rt / r);
    return 2.0 * R + sqrt(2.0 * L * (vhat + 4.0 * R) / r) + L / (3.0 * r);
}
static double xi0(double vhat, double r, double delta) {
    const double L = log(4.0 / delta);
    return sqrt(2.0 * L * vhat / r) + L / (3.0 * r);
}
static int64_t hoeffding(int64_t n, double eps, double delta) {
    return (int64_t)ceil(log(2.0 * (double)n / delta) / (2.0 * eps * eps));
}
static int64_t omega(double vhat, double rho, double eps, double delta, int64_t n) {
    if (vhat <= 0.0 || rho <= 0.0) return hoeffding(n, eps, delta);
    double x = (2.0 * vhat + 2.0 * eps / 3.0) / (eps * eps) * (log(2.0 * rho / vhat) + log(1.0 / delta));
    return (int64_t)ceil(x);
}
static int64_t boot(double eps, double delta) { return (int64_t)ceil(log(1.0 / delta) / eps); }
static int64_t first(int64_t sb, int64_t om, double vhat, double eps, double d1) {
    int64_t lo = sb, hi = om;
    if (xi0(vhat, (double)hi, d1) > eps) return hi;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (xi0(vhat, (double)mid, d1) <= eps) hi = mid; else lo = mid + 1;
    }
    return lo;
}
static int64_t next(int64_t prev) {
    int64_t x = (6 * prev + 4) / 5;
    return x > prev ? x : prev + 1;
}
}  // namespace bnd

// ------------------------------------------------------------------ graph

struct SlabPool {
    int nslabs = 0;
    int64_t nmax = 0, cap = 0, gmax = 0;
    u64 *F = nullptr, *R = nullptr, *N = nullptr, *AG = nullptr, *arcs = nullptr, *XS = nullptr;
    u32 *AGF = nullptr, *hdr = nullptr;
    int32_t *touched = nullptr;
    void release() {
        hipFree(F); hipFree(R); hipFree(N); hipFree(AG); hipFree(arcs); hipFree(XS);
        hipFree(AGF); hipFree(hdr); hipFree(touched);
        F = R = N = AG = arcs = XS = nullptr;
        AGF = hdr = nullptr;
        touched = nullptr;
        nslabs = 0;
    }
    DevSlabs view() const {
        DevSlabs s;
        s.F = F; s.R = R; s.N = N; s.AG = AG; s.AGF = AGF; s.touched = touched; s.arcs = arcs;
        s.XS = XS; s.hdr = hdr; s.nmax = nmax; s.cap = cap; s.gmax = gmax;
        return s;
    }
};

struct ServeState;

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
    int64_t *dout_off = nullptr, *din_off = nullptr, *dseg_eoff = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    SlabPool pool, pool_big;
    int user_slabs = 0;
    int64_t user_cap = 0;
    // misc device buffers
    u32 *dwork = nullptr;
    u64 *dstats = nullptr;
    int32_t *dretry = nullptr;
    int64_t retry_cap = 0;
    double *dpart = nullptr;
    int part_blocks = 0, part_c = -1;
    DevReq *dreqs = nullptr;
    int dreq_cap = 0;
    std::mutex mu;  // one blocking call at a time per graph
    // timing of the last blocking call
    double last_ms = 0;
    int64_t last_launches = 0, last_W = 0, last_arcs = 0, last_tn = 0, last_te = 0;
    ServeState *serve = nullptr;
    DevGraph dev() const {
        DevGraph d;
        d.U = dU; d.V = dV; d.T = dT; d.out_off = dout_off; d.out_t = dout_t; d.in_off = din_off;
        d.in_t = din_t; d.seg_eoff = dseg_eoff; d.seg_noff = dseg_noff; d.n_total = n_total;
        d.G = G; d.m = m; d.perm = dperm;
        return d;
    }
};

static int pick_device(int *dev) {
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess || cnt <= 0) return fail(MANTRA_E_NODEV, "no HIP device");
    int d = 0;
    hipGetDevice(&d);
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, d) != hipSuccess) return fail(MANTRA_E_NODEV, "no device properties");
    if (strncmp(pr.gcnArchName, "gfx950", 6) != 0)
        return fail(MANTRA_E_NODEV, "device %d is %s, this library is built for gfx950", d, pr.gcnArchName);
    *dev = d;
    return MANTRA_OK;
}

struct EdgeRec { int32_t g, t, v, u; int64_t idx; };

static int build_graph(int32_t G, const int32_t *node_count, const int64_t *edge_off,
                       const int32_t *src, const int32_t *dst, const int32_t *t, mantra_graph **out) {
    if (!out) return fail(MANTRA_E_INVALID, "out is NULL");
    *out = nullptr;
    if (G < 1) return fail(MANTRA_E_INVALID, "need at least one graph");
    int64_t m = edge_off[G];
    if (m < 0) return fail(MANTRA_E_INVALID, "negative edge count");
    if (m > 0 && (!src || !dst || !t)) return fail(MANTRA_E_INVALID, "edge arrays are NULL");
    if (m >= (int64_t)1 << 32) return fail(MANTRA_E_INVALID, "at most 2^32-1 edges");
    std::unique_ptr<mantra_graph> g(new mantra_graph());
    int rc = pick_device(&g->device);
    if (rc) return rc;
    g->G = G;
    g->m_in = m;
    g->seg_noff.assign(G + 1, 0);
    int64_t ntot = 0;
    int32_t nmax = 0;
    for (int i = 0; i < G; ++i) {
        if (node_count[i] < 2) return fail(MANTRA_E_INVALID, "graph %d has fewer than 2 nodes", i);
        if (edge_off[i + 1] < edge_off[i]) return fail(MANTRA_E_INVALID, "edge offsets decrease at %d", i);
        g->seg_noff[i] = (int32_t)ntot;
        ntot += node_count[i];
        if (node_count[i] > nmax) nmax = node_count[i];
        if (ntot >= INT32_MAX) return fail(MANTRA_E_INVALID, "too many nodes");
    }
    if (edge_off[0] != 0) return fail(MANTRA_E_INVALID, "edge_off[0] must be 0");
    g->seg_noff[G] = (int32_t)ntot;
    g->n_total = (int32_t)ntot;
    g->nmax = nmax;
    // internal node ids: each graph's nodes ordered by total degree, highest
    // first, so that the per-pair state of the hubs (which most edges touch
    // in skewed graphs) shares a few cache lines
    {
        std::vector<int64_t> deg((size_t)ntot, 0);
        for (int gi = 0; gi < G; ++gi) {
            int32_t ng = node_count[gi];
            for (int64_t i = edge_off[gi]; i < edge_off[gi + 1]; ++i) {
                int32_t u = src[i], v = dst[i];
                if (u >= 0 && u < ng) deg[(size_t)(g->seg_noff[gi] + u)]++;
                if (v >= 0 && v < ng) deg[(size_t)(g->seg_noff[gi] + v)]++;
            }
        }
        g->perm.assign((size_t)ntot, 0);
        g->iperm.assign((size_t)ntot, 0);
        std::vector<int32_t> ord;
        for (int gi = 0; gi < G; ++gi) {
            int32_t b = g->seg_noff[gi], ng = node_count[gi];
            ord.resize((size_t)ng);
            for (int32_t i = 0; i < ng; ++i) ord[(size_t)i] = b + i;
            std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return deg[(size_t)x] > deg[(size_t)y]; });
            for (int32_t i = 0; i < ng; ++i) {
                g->perm[(size_t)ord[(size_t)i]] = b + i;
                g->iperm[(size_t)(b + i)] = ord[(size_t)i];
            }
        }
    }
    std::vector<EdgeRec> E((size_t)m);
    for (int gi = 0; gi < G; ++gi) {
        int32_t ng = node_count[gi];
        for (int64_t i = edge_off[gi]; i < edge_off[gi + 1]; ++i) {
            int32_t u = src[i], v = dst[i], tt = t[i];
            if (u < 0 || u >= ng || v < 0 || v >= ng)
                return fail(MANTRA_E_INVALID, "edge %lld: node id outside [0, %d)", (long long)i, ng);
            if (u == v) return fail(MANTRA_E_INVALID, "edge %lld: self-loop on %d", (long long)i, u);
            if (tt < 0 || tt == INT32_MAX)
                return fail(MANTRA_E_INVALID, "edge %lld: time %d outside [0, 2^31-2]", (long long)i, tt);
            int32_t b = g->seg_noff[gi];
            E[(size_t)i] = EdgeRec{gi, tt, g->perm[(size_t)(b + v)] - b, g->perm[(size_t)(b + u)] - b, i};
        }
    }
    std::sort(E.begin(), E.end(), [](const EdgeRec &a, const EdgeRec &b) {
        if (a.g != b.g) return a.g < b.g;
        if (a.t != b.t) return a.t < b.t;
        if (a.v != b.v) return a.v < b.v;
        if (a.u != b.u) return a.u < b.u;
        return a.idx < b.idx;
    });
    g->in2k.assign((size_t)m, -1);
    std::vector<int32_t> U, V, T;
    U.reserve((size_t)m); V.reserve((size_t)m); T.reserve((size_t)m);
    g->seg_eoff.assign(G + 1, 0);
    int64_t k = -1;
    for (size_t i = 0; i < E.size(); ++i) {
        const EdgeRec &e = E[i];
        bool dup = i > 0 && E[i - 1].g == e.g && E[i - 1].t == e.t && E[i - 1].v == e.v && E[i - 1].u == e.u;
        if (!dup) {
            ++k;
            U.push_back(e.u); V.push_back(e.v); T.push_back(e.t);
            g->seg_eoff[e.g + 1] = k + 1;
        } else {
            g->ndup++;
        }
        g->in2k[(size_t)e.idx] = k;
    }
    for (int gi = 0; gi < G; ++gi)
        if (g->seg_eoff[gi + 1] < g->seg_eoff[gi]) g->seg_eoff[gi + 1] = g->seg_eoff[gi];
    const int64_t mu = (int64_t)U.size();
    g->m = mu;
    E.clear();
    E.shrink_to_fit();
    g->tmin = mu ? *std::min_element(T.begin(), T.end()) : 0;
    g->tmax = mu ? *std::max_element(T.begin(), T.end()) : 0;
    // largest tick (edges sharing a time in one graph)
    int64_t run = 0, gm = 1;
    for (int64_t i = 0; i < mu; ++i) {
        bool same = i > 0 && T[i] == T[i - 1];
        if (same) {
            // same graph? segments are contiguous: check the segment boundary
            int gi = (int)(std::upper_bound(g->seg_eoff.begin(), g->seg_eoff.end(), i) - g->seg_eoff.begin()) - 1;
            same = i > g->seg_eoff[gi];
        }
        run = same ? run + 1 : 1;
        if (run > gm) gm = run;
    }
    g->gmax = gm;
    // CSR of out- and in-edge times per global node (ascending times)
    std::vector<int64_t> ooff((size_t)ntot + 1, 0), ioff((size_t)ntot + 1, 0);
    std::vector<int32_t> ot((size_t)(mu ? mu : 1)), it((size_t)(mu ? mu : 1));
    for (int gi = 0; gi < G; ++gi)
        for (int64_t i = g->seg_eoff[gi]; i < g->seg_eoff[gi + 1]; ++i) {
            ooff[(size_t)(g->seg_noff[gi] + U[i]) + 1]++;
            ioff[(size_t)(g->seg_noff[gi] + V[i]) + 1]++;
        }
    for (int64_t v = 0; v < ntot; ++v) { ooff[v + 1] += ooff[v]; ioff[v + 1] += ioff[v]; }
    {
        std::vector<int64_t> co(ooff.begin(), ooff.end() - 1), ci(ioff.begin(), ioff.end() - 1);
        for (int gi = 0; gi < G; ++gi)
            for (int64_t i = g->seg_eoff[gi]; i < g->seg_eoff[gi + 1]; ++i) {
                ot[(size_t)co[g->seg_noff[gi] + U[i]]++] = T[i];
                it[(size_t)ci[g->seg_noff[gi] + V[i]]++] = T[i];
            }
    }
    hipSetDevice(g->device);
    HIPCHK(dalloc(&g->dU, mu));
    HIPCHK(dalloc(&g->dV, mu));
    HIPCHK(dalloc(&g->dT, mu));
    HIPCHK(dalloc(&g->dout_t, mu));
    HIPCHK(dalloc(&g->din_t, mu));
    HIPCHK(dalloc(&g->dout_off, ntot + 1));
    HIPCHK(dalloc(&g->din_off, ntot + 1));
    HIPCHK(dalloc(&g->dseg_eoff, G + 1));
    HIPCHK(dalloc(&g->dseg_noff, G + 1));
    HIPCHK(dalloc(&g->dperm, ntot));
    HIPCHK(hipMemcpy(g->dperm, g->perm.data(), sizeof(int32_t) * ntot, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->dU, U.data(), sizeof(int32_t) * mu, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->dV, V.data(), sizeof(int32_t) * mu, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->dT, T.data(), sizeof(int32_t) * mu, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->dout_t, ot.data(), sizeof(int32_t) * mu, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->din_t, it.data(), sizeof(int32_t) * mu, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->dout_off, ooff.data(), sizeof(int64_t) * (ntot + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->din_off, ioff.data(), sizeof(int64_t) * (ntot + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->dseg_eoff, g->seg_eoff.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->dseg_noff, g->seg_noff.data(), sizeof(int32_t) * (G + 1), hipMemcpyHostToDevice));
    HIPCHK(hipStreamCreate(&g->st));
    HIPCHK(hipEventCreate(&g->ev0));
    HIPCHK(hipEventCreate(&g->ev1));
    HIPCHK(dalloc(&g->dwork, 1));
    HIPCHK(dalloc(&g->dstats, 16));
    *out = g.release();
    return MANTRA_OK;
}

// ------------------------------------------------------------------ slabs

// A reached-bitmap in LDS lets a batch skip the state loads of unreached
// tails; beyond 8 KB it costs more occupancy than it saves, and the reached
// test reads the gathered per-node state (its pair tag) instead.
static int lds_bitmap_ok(int64_t nmax) { return ((nmax + 31) / 32) * 4 <= 8 * 1024; }
static size_t lds_bytes(int64_t nmax) {
    size_t b = mantra_tab_lds_bytes();
    if (lds_bitmap_ok(nmax)) b += (size_t)((nmax + 31) / 32) * 4;
    else b += (size_t)kAliveN * 4;  // alive-set hash of the reverse sweep
    return b;
}

static int auto_slabs(const mantra_graph *g) {
    if (g->user_slabs > 0) return g->user_slabs;
    hipDeviceProp_t pr;
    hipGetDeviceProperties(&pr, g->device);
    int cus = pr.multiProcessorCount > 0 ? pr.multiProcessorCount : 256;
    // resident workgroups per CU (registers and LDS), as the runtime reports
    size_t lb = lds_bytes(g->nmax);
    int per_cu = mantra_sweep_occupancy(lb);
    if (per_cu <= 0) {
        int by_lds = (int)((160 * 1024) / (lb ? lb : 1));
        per_cu = std::min(8, std::max(1, by_lds));
    }
    return cus * per_cu;
}

static int pool_ensure(mantra_graph *g, SlabPool &p, int nslabs, int64_t cap) {
    int64_t nmax = g->nmax;
    int64_t gmax = g->gmax;
    if (p.nslabs >= nslabs && p.cap >= cap && p.nmax == nmax && p.gmax >= gmax) return MANTRA_OK;
    p.release();
    p.nmax = nmax; p.cap = cap; p.gmax = gmax;
    size_t ns = (size_t)nslabs;
    if (dalloc(&p.F, ns * nmax * 2) || dalloc(&p.R, ns * nmax * 2) || dalloc(&p.N, ns * nmax) ||
        dalloc(&p.AG, ns * nmax * 2) || dalloc(&p.AGF, ns * nmax) || dalloc(&p.touched, ns * nmax) ||
        dalloc(&p.arcs, ns * (size_t)cap * 4) || dalloc(&p.XS, ns * (size_t)gmax * 2) ||
        dalloc(&p.hdr, ns * 4)) {
        p.release();
        (void)hipGetLastError();
        return fail(MANTRA_E_OOM, "slab pool: %d slabs x (%lld nodes, %lld arcs) does not fit", nslabs,
                    (long long)nmax, (long long)cap);
    }
    HIPCHK(hipMemsetAsync(p.F, 0, sizeof(u64) * ns * nmax * 2, g->st));
    HIPCHK(hipMemsetAsync(p.R, 0, sizeof(u64) * ns * nmax * 2, g->st));
    HIPCHK(hipMemsetAsync(p.N, 0, sizeof(u64) * ns * nmax, g->st));
    HIPCHK(hipMemsetAsync(p.AG, 0xFF, sizeof(u64) * ns * nmax * 2, g->st));
    HIPCHK(hipMemsetAsync(p.AGF, 0, sizeof(u32) * ns * nmax, g->st));
    HIPCHK(hipMemsetAsync(p.hdr, 0, sizeof(u32) * ns * 4, g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    p.nslabs = nslabs;
    return MANTRA_OK;
}

static int64_t auto_cap(const mantra_graph *g, int nslabs) {
    if (g->user_cap > 0) return g->user_cap;
    size_t fr = 0, tot = 0;
    hipMemGetInfo(&fr, &tot);
    // arcs take at most a quarter of free memory; 16 bytes each
    int64_t per = (int64_t)(fr / 4 / 16 / (size_t)std::max(1, nslabs));
    int64_t cap = std::min<int64_t>(g->m + 1, std::max<int64_t>(per, 1 << 16));
    return std::max<int64_t>(cap, 1024);
}

// ------------------------------------------------------------------ launches

struct LaunchSpec {
    std::vector<DevReq> reqs;
    int64_t npairs = 0;
    const int32_t *dpg = nullptr, *dps = nullptr, *dpz = nullptr;
    void *drec = nullptr;
    double *dnode_f = nullptr, *dedge_f = nullptr;
};

// launch the sweep over all pairs of spec; re-run pairs whose arcs did not
// fit with a pool of few slabs and the largest capacity.  Adds the device
// time of the sweep launches to g->last_ms.
static int run_sweep(mantra_graph *g, const LaunchSpec &sp, u64 stats_out[16]) {
    if (sp.npairs <= 0) { memset(stats_out, 0, sizeof(u64) * 16); return MANTRA_OK; }
    hipSetDevice(g->device);
    int ns = auto_slabs(g);
    if ((int64_t)ns > sp.npairs) ns = (int)sp.npairs;
    int64_t cap = auto_cap(g, auto_slabs(g));
    int rc = pool_ensure(g, g->pool, std::max(ns, g->pool.nslabs), std::max(cap, g->pool.cap));
    if (rc) return rc;
    if ((int)sp.reqs.size() > g->dreq_cap) {
        hipFree(g->dreqs);
        g->dreqs = nullptr;
        g->dreq_cap = std::max<int>(64, (int)sp.reqs.size());
        HIPCHK(dalloc(&g->dreqs, (size_t)g->dreq_cap));
    }
    if (sp.npairs + 1 > g->retry_cap) {
        hipFree(g->dretry);
        g->retry_cap = std::max<int64_t>(sp.npairs + 1, 4096);
        HIPCHK(dalloc(&g->dretry, (size_t)g->retry_cap));
    }
    HIPCHK(hipMemcpyAsync(g->dreqs, sp.reqs.data(), sizeof(DevReq) * sp.reqs.size(), hipMemcpyHostToDevice, g->st));
    HIPCHK(hipMemsetAsync(g->dwork, 0, sizeof(u32), g->st));
    HIPCHK(hipMemsetAsync(g->dstats, 0, sizeof(u64) * 16, g->st));
    HIPCHK(hipMemsetAsync(g->dretry, 0, sizeof(int32_t), g->st));
    LaunchArgs a;
    memset(&a, 0, sizeof a);
    a.g = g->dev();
    a.sl = g->pool.view();
    a.reqs = g->dreqs;
    a.nreq = (int32_t)sp.reqs.size();
    a.lds_bitmap = lds_bitmap_ok(g->nmax);
    a.npairs = sp.npairs;
    a.pg = sp.dpg; a.ps = sp.dps; a.pz = sp.dpz; a.pq = nullptr;
    a.rec = sp.drec;
    a.node_f = sp.dnode_f;
    a.edge_f = sp.dedge_f;
    a.work = g->dwork;
    a.stats = g->dstats;
    a.retry = g->dretry;
    size_t lb = lds_bytes(g->nmax);
    HIPCHK(hipEventRecord(g->ev0, g->st));
    HIPCHK(mantra_launch_sweep(&a, ns, lb, g->st));
    HIPCHK(hipEventRecord(g->ev1, g->st));
    int32_t nretry = 0;
    HIPCHK(hipMemcpyAsync(&nretry, g->dretry, sizeof(int32_t), hipMemcpyDeviceToHost, g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
    g->last_ms += ms;
    g->last_launches += 1;
    u64 st1[16];
    HIPCHK(hipMemcpy(st1, g->dstats, sizeof(u64) * 16, hipMemcpyDeviceToHost));
    if (nretry > 0) {
        // pairs whose appearance-DAG arcs exceeded the slab capacity
        int ns2 = std::min<int>(nretry, 64);
        int64_t cap2 = g->m + 1;
        rc = pool_ensure(g, g->pool_big, ns2, cap2);
        if (rc) return rc;
        std::vector<int32_t> q((size_t)nretry + 1);
        HIPCHK(hipMemcpy(q.data(), g->dretry, sizeof(int32_t) * (nretry + 1), hipMemcpyDeviceToHost));
        int32_t *dq = nullptr;
        HIPCHK(dalloc(&dq, (size_t)nretry));
        HIPCHK(hipMemcpy(dq, q.data() + 1, sizeof(int32_t) * nretry, hipMemcpyHostToDevice));
        HIPCHK(hipMemsetAsync(g->dwork, 0, sizeof(u32), g->st));
        HIPCHK(hipMemsetAsync(g->dstats, 0, sizeof(u64) * 16, g->st));
        HIPCHK(hipMemsetAsync(g->dretry, 0, sizeof(int32_t), g->st));
        a.sl = g->pool_big.view();
        a.npairs = nretry;
        a.pq = dq;
        HIPCHK(hipEventRecord(g->ev0, g->st));
        HIPCHK(mantra_launch_sweep(&a, ns2, lb, g->st));
        HIPCHK(hipEventRecord(g->ev1, g->st));
        HIPCHK(hipStreamSynchronize(g->st));
        HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
        g->last_ms += ms;
        g->last_launches += 1;
        u64 st2[16];
        HIPCHK(hipMemcpy(st2, g->dstats, sizeof(u64) * 16, hipMemcpyDeviceToHost));
        hipFree(dq);
        int32_t n2 = 0;
        HIPCHK(hipMemcpy(&n2, g->dretry, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (n2 > 0) return fail(MANTRA_E_INTERNAL, "arc buffer of a full window overflowed");
        for (int i = 0; i < 16; ++i)
            if (i != 5) st1[i] += st2[i];
    }
    memcpy(stats_out, st1, sizeof(st1));
    g->last_W += (int64_t)st1[0];
    g->last_arcs += (int64_t)st1[1];
    g->last_tn += (int64_t)st1[7];
    g->last_te += (int64_t)st1[8];
    if (st1[6]) return fail(MANTRA_E_INTERNAL, "%llu pairs failed flow conservation", (unsigned long long)st1[6]);
    return MANTRA_OK;
}

// per-block partials of max W, sum B, max R_j
static int reduce(mantra_graph *g, const double *W, const double *B, const double *R, int64_t n, int c,
                  double *maxW, double *sumB, std::vector<double> &maxR) {
    int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
    if (g->part_blocks < blocks || g->part_c < c) {
        hipFree(g->dpart);
        g->dpart = nullptr;
        g->part_blocks = 1024;
        g->part_c = std::max(c, 64);
        HIPCHK(dalloc(&g->dpart, (size_t)1024 * (2 + g->part_c)));
    }
    ReduceArgs ra;
    ra.W = W; ra.B = B; ra.R = R; ra.n = n; ra.c = c; ra.part = g->dpart;
    HIPCHK(mantra_launch_reduce(&ra, blocks, g->st));
    std::vector<double> part((size_t)blocks * (2 + c));
    HIPCHK(hipMemcpyAsync(part.data(), g->dpart, sizeof(double) * part.size(), hipMemcpyDeviceToHost, g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    double mw = -INFINITY, sb = 0.0;
    maxR.assign((size_t)c, -INFINITY);
    for (int b = 0; b < blocks; ++b) {
        const double *p = &part[(size_t)b * (2 + c)];
        mw = std::max(mw, p[0]);
        sb += p[1];
        for (int j = 0; j < c; ++j) maxR[(size_t)j] = std::max(maxR[(size_t)j], p[2 + j]);
    }
    *maxW = mw;
    *sumB = sb;
    return MANTRA_OK;
}

// ------------------------------------------------------------------ requests

struct Acc {
    double *B = nullptr, *W = nullptr, *R = nullptr, *E = nullptr;
    int64_t n = 0, m = 0;
    int c = 0;
    void release() { hipFree(B); hipFree(W); hipFree(R); hipFree(E); B = W = R = E = nullptr; }
};

static int acc_alloc(mantra_graph *g, Acc &a, int c, bool edges) {
    a.n = g->n_total; a.m = g->m; a.c = c;
    HIPCHK(dalloc(&a.B, (size_t)a.n));
    HIPCHK(dalloc(&a.W, (size_t)a.n));
    HIPCHK(dalloc(&a.R, (size_t)a.n * (size_t)std::max(c, 1)));
    if (edges) HIPCHK(dalloc(&a.E, (size_t)a.m));
    return MANTRA_OK;
}
static int acc_zero(mantra_graph *g, Acc &a) {
    HIPCHK(hipMemsetAsync(a.B, 0, sizeof(double) * a.n, g->st));
    HIPCHK(hipMemsetAsync(a.W, 0, sizeof(double) * a.n, g->st));
    HIPCHK(hipMemsetAsync(a.R, 0, sizeof(double) * a.n * std::max(a.c, 1), g->st));
    if (a.E) HIPCHK(hipMemsetAsync(a.E, 0, sizeof(double) * a.m, g->st));
    return MANTRA_OK;
}

static DevReq make_req(const mantra_request &rq, int stream, int64_t base, int64_t qoff, int64_t count,
                       const Acc &acc, int c) {
    DevReq d;
    memset(&d, 0, sizeof d);
    d.opt = rq.opt;
    d.t0 = rq.t0;
    d.t1 = rq.t1;
    d.c = c;
    d.seed = rq.seed;
    d.stream = stream;
    d.graph = 0;
    d.base = base;
    d.qoff = qoff;
    d.count = count;
    d.per_graph = count;
    d.Bsum = acc.B;
    d.Wsum = acc.W;
    d.Rsum = c > 0 ? acc.R : nullptr;
    d.Esum = acc.E;
    return d;
}

static int check_request(const mantra_graph *g, const mantra_request &rq) {
    if (rq.opt < MANTRA_SH || rq.opt > MANTRA_PFM) return fail(MANTRA_E_INVALID, "unknown optimality %d", (int)rq.opt);
    if (!rq.node_bc) return fail(MANTRA_E_INVALID, "node_bc is NULL");
    int c = rq.c ? rq.c : 25;
    if (c < 1 || c > 64) return fail(MANTRA_E_INVALID, "c = %d outside 1..64", c);
    if (rq.fixed_r <= 0) {
        if (!(rq.eps > 0 && rq.eps < 1)) return fail(MANTRA_E_INVALID, "eps must be in (0, 1)");
        if (!(rq.delta > 0 && rq.delta < 1)) return fail(MANTRA_E_INVALID, "delta must be in (0, 1)");
        if (g->G != 1) return fail(MANTRA_E_INVALID, "progressive sampling needs a single graph; use fixed_r");
    } else if (rq.fixed_r > ((int64_t)1 << 40)) {
        return fail(MANTRA_E_INVALID, "fixed_r too large");
    }
    return MANTRA_OK;
}

static void norm_window(mantra_request &rq) {
    if (rq.t1 < rq.t0) { rq.t0 = 0; rq.t1 = INT32_MAX; }
}

static int finish_outputs(mantra_graph *g, const mantra_request &rq, Acc &acc, int64_t r) {
    std::vector<double> hb((size_t)g->n_total);
    HIPCHK(hipMemcpyAsync(hb.data(), acc.B, sizeof(double) * g->n_total, hipMemcpyDeviceToHost, g->st));
    std::vector<double> he;
    if (rq.edge_bc && acc.E) {
        he.resize((size_t)g->m);
        HIPCHK(hipMemcpyAsync(he.data(), acc.E, sizeof(double) * g->m, hipMemcpyDeviceToHost, g->st));
    }
    HIPCHK(hipStreamSynchronize(g->st));
    double rr = (double)r;
    for (int64_t v = 0; v < g->n_total; ++v) rq.node_bc[g->iperm[(size_t)v]] = r ? hb[(size_t)v] / rr : 0.0;
    if (rq.edge_bc && acc.E)
        for (int64_t i = 0; i < g->m_in; ++i) rq.edge_bc[i] = r ? he[(size_t)g->in2k[(size_t)i]] / rr : 0.0;
    return MANTRA_OK;
}

// Algorithm 1 (or a fixed sample) for one request, blocking
static int run_request(mantra_graph *g, mantra_request rq, mantra_result *res) {
    auto t_start = std::chrono::steady_clock::now();
    int rc = check_request(g, rq);
    if (rc) return rc;
    norm_window(rq);
    const int c = rq.c ? rq.c : 25;
    const bool edges = (rq.flags & MANTRA_F_EDGE_BC) && rq.edge_bc;
    mantra_result R;
    memset(&R, 0, sizeof R);
    if (rq.opt == MANTRA_FM) R.flags |= MANTRA_RES_NO_GUARANTEE;
    g->last_ms = 0; g->last_launches = 0; g->last_W = 0; g->last_arcs = 0; g->last_tn = 0; g->last_te = 0;
    Acc acc;
    rc = acc_alloc(g, acc, c, edges);
    if (rc) { acc.release(); return rc; }
    rc = acc_zero(g, acc);
    u64 st[16];
    int64_t r = 0;
    if (!rc && rq.fixed_r > 0) {
        LaunchSpec sp;
        int64_t npairs = rq.fixed_r * g->G;
        DevReq d = make_req(rq, STREAM_PAIR, 0, 0, npairs, acc, c);
        d.graph = g->G == 1 ? 0 : -1;
        d.per_graph = rq.fixed_r;
        sp.reqs.push_back(d);
        sp.npairs = npairs;
        rc = run_sweep(g, sp, st);
        if (!rc) {
            r = rq.fixed_r;
            R.samples = r;
            R.rounds = 1;
            R.n_overflow = (int64_t)st[2];
            R.n_reachable = (int64_t)st[3];
            if (st[4]) rc = fail(MANTRA_E_LIMIT, "a hop count exceeded 65534");
        }
        if (!rc && g->G == 1) {
            double mw, sb;
            std::vector<double> mr;
            rc = reduce(g, acc.W, acc.B, acc.R, g->n_total, c, &mw, &sb, mr);
            if (!rc) {
                double W = std::max(mw, 0.0) / (double)r, Rc = 0;
                for (int j = 0; j < c; ++j) Rc += mr[(size_t)j] / (double)r;
                Rc /= c;
                R.wimpy = W;
                R.mcera = Rc;
                R.xi = bnd::xi(Rc, W, std::min(0.25, W), c, (double)r, rq.delta > 0 && rq.delta < 1 ? rq.delta : 0.1);
            }
        }
    } else if (!rc) {
        // bootstrap: s' pairs of the BOOT stream (delta/2 of the budget)
        const int64_t sb = bnd::boot(rq.eps, rq.delta);
        R.s_boot = sb;
        Acc boot;
        rc = acc_alloc(g, boot, 0, false);
        if (!rc) rc = acc_zero(g, boot);
        if (!rc) {
            LaunchSpec sp;
            sp.reqs.push_back(make_req(rq, STREAM_BOOT, 0, 0, sb, boot, 0));
            sp.npairs = sb;
            rc = run_sweep(g, sp, st);
            if (!rc && st[4]) rc = fail(MANTRA_E_LIMIT, "a hop count exceeded 65534");
            if (!rc && st[2]) { R.n_overflow += (int64_t)st[2]; }
        }
        double mw = 0, sumb = 0;
        std::vector<double> mr;
        if (!rc) rc = reduce(g, boot.W, boot.B, boot.R, g->n_total, 0, &mw, &sumb, mr);
        boot.release();
        int64_t om = 0, s1 = 0;
        if (!rc) {
            R.rho_hat = sumb / (double)sb;
            double wb = std::max(mw, 0.0) / (double)sb;
            R.v_hat = std::min(0.25, wb);
            om = std::max<int64_t>(sb, bnd::omega(R.v_hat, R.rho_hat, rq.eps, rq.delta / 2.0, g->n_total));
            if (rq.max_samples > 0) om = std::min(om, rq.max_samples);
            s1 = rq.s1 > 0 ? rq.s1 : bnd::first(sb, om, R.v_hat, rq.eps, rq.delta / 4.0);
            s1 = std::min(s1, om);
            R.omega = om;
            R.s1 = s1;
        }
        int64_t prev = 0;
        int i = 0;
        while (!rc) {
            ++i;
            int64_t si = (i == 1) ? s1 : std::min(bnd::next(prev), om);
            LaunchSpec sp;
            sp.reqs.push_back(make_req(rq, STREAM_PAIR, prev, 0, si - prev, acc, c));
            sp.npairs = si - prev;
            rc = run_sweep(g, sp, st);
            if (rc) break;
            R.n_overflow += (int64_t)st[2];
            R.n_reachable += (int64_t)st[3];
            if (st[4]) { rc = fail(MANTRA_E_LIMIT, "a hop count exceeded 65534"); break; }
            double sumB;
            rc = reduce(g, acc.W, acc.B, acc.R, g->n_total, c, &mw, &sumB, mr);
            if (rc) break;
            r = si;
            double W = std::max(mw, 0.0) / (double)r, Rc = 0;
            for (int j = 0; j < c; ++j) Rc += mr[(size_t)j] / (double)r;
            Rc /= c;
            double di = rq.delta / pow(2.0, (double)(i + 1));
            double xi = bnd::xi(Rc, W, std::min(0.25, W), c, (double)r, di);
            R.xi = xi; R.wimpy = W; R.mcera = Rc; R.rounds = i; R.samples = r;
            if (r >= om) { R.flags |= MANTRA_RES_STOP_OMEGA; break; }
            if (xi <= rq.eps) { R.flags |= MANTRA_RES_STOP_XI; break; }
            prev = si;
        }
    }
    if (!rc) rc = finish_outputs(g, rq, acc, r);
    acc.release();
    if (!rc && R.n_overflow > 0) rc = fail(MANTRA_E_OVERFLOW, "%lld sampled pairs saturated", (long long)R.n_overflow);
    R.window_edges = g->last_W;
    R.arcs = g->last_arcs;
    R.gpu_ms = g->last_ms;
    R.latency_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    R.status = rc;
    if (rc == MANTRA_E_OVERFLOW)
        for (int64_t v = 0; v < g->n_total; ++v) rq.node_bc[v] = NAN;
    if (res) *res = R;
    return rc;
}

// ------------------------------------------------------------------ C ABI

extern "C" {

const char *mantra_last_error(void) { return g_err.c_str(); }

int mantra_graph_create(const int32_t *src, const int32_t *dst, const int32_t *t, int64_t m, int32_t n,
                        uint32_t flags, mantra_graph **out) {
    (void)flags;
    int64_t off[2] = {0, m};
    int32_t nc[1] = {n};
    return build_graph(1, nc, off, src, dst, t, out);
}

int mantra_graph_create_packed(int32_t G, const int32_t *node_count, const int64_t *edge_off,
                               const int32_t *src, const int32_t *dst, const int32_t *t, uint32_t flags,
                               mantra_graph **out) {
    (void)flags;
    if (!node_count || !edge_off) return fail(MANTRA_E_INVALID, "node_count / edge_off NULL");
    return build_graph(G, node_count, edge_off, src, dst, t, out);
}

int mantra_serve_stop(mantra_graph *g);

void mantra_graph_destroy(mantra_graph *g) {
    if (!g) return;
    mantra_serve_stop(g);
    hipSetDevice(g->device);
    if (g->st) hipStreamSynchronize(g->st);
    g->pool.release();
    g->pool_big.release();
    hipFree(g->dU); hipFree(g->dV); hipFree(g->dT); hipFree(g->dout_t); hipFree(g->din_t);
    hipFree(g->dout_off); hipFree(g->din_off); hipFree(g->dseg_eoff); hipFree(g->dseg_noff); hipFree(g->dperm);
    hipFree(g->dwork); hipFree(g->dstats); hipFree(g->dretry); hipFree(g->dpart); hipFree(g->dreqs);
    if (g->ev0) hipEventDestroy(g->ev0);
    if (g->ev1) hipEventDestroy(g->ev1);
    if (g->st) hipStreamDestroy(g->st);
    delete g;
}

int mantra_graph_info(const mantra_graph *g, int32_t *n, int64_t *m_unique, int64_t *n_duplicates,
                      int32_t *t_min, int32_t *t_max, int32_t *n_graphs) {
    if (!g) return fail(MANTRA_E_INVALID, "graph is NULL");
    if (n) *n = g->n_total;
    if (m_unique) *m_unique = g->m;
    if (n_duplicates) *n_duplicates = g->ndup;
    if (t_min) *t_min = g->tmin;
    if (t_max) *t_max = g->tmax;
    if (n_graphs) *n_graphs = g->G;
    return MANTRA_OK;
}

int mantra_set_launch(mantra_graph *g, int32_t n_slabs, int64_t arc_cap) {
    if (!g) return fail(MANTRA_E_INVALID, "graph is NULL");
    if (n_slabs < 0 || arc_cap < 0) return fail(MANTRA_E_INVALID, "negative launch setting");
    std::lock_guard<std::mutex> lk(g->mu);
    g->user_slabs = n_slabs;
    g->user_cap = arc_cap;
    g->pool.release();
    return MANTRA_OK;
}

int mantra_last_timing(const mantra_graph *g, double *sweep_ms, int64_t *launches, int64_t *window_edges,
                       int64_t *arcs, int64_t *touched_nodes, int64_t *touched_edges) {
    if (!g) return fail(MANTRA_E_INVALID, "graph is NULL");
    g_err.clear();
    if (sweep_ms) *sweep_ms = g->last_ms;
    if (launches) *launches = g->last_launches;
    if (window_edges) *window_edges = g->last_W;
    if (arcs) *arcs = g->last_arcs;
    if (touched_nodes) *touched_nodes = g->last_tn;
    if (touched_edges) *touched_edges = g->last_te;
    return MANTRA_OK;
}

int mantra_count_pairs(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r,
                       const int32_t *graph, const int32_t *s, const int32_t *z, mantra_pair_record *out,
                       double *node_f, double *edge_f) {
    if (!g) return fail(MANTRA_E_INVALID, "graph is NULL");
    if (r < 0 || (r > 0 && (!s || !z || !out))) return fail(MANTRA_E_INVALID, "bad pair arrays");
    if (opt < MANTRA_SH || opt > MANTRA_PFM) return fail(MANTRA_E_INVALID, "unknown optimality %d", (int)opt);
    if (r == 0) return MANTRA_OK;
    if (r > INT32_MAX) return fail(MANTRA_E_INVALID, "too many pairs");
    for (int64_t q = 0; q < r; ++q) {
        int32_t gi = graph ? graph[q] : 0;
        if (gi < 0 || gi >= g->G) return fail(MANTRA_E_INVALID, "pair %lld: graph %d", (long long)q, gi);
        int32_t ng = g->seg_noff[gi + 1] - g->seg_noff[gi];
        if (s[q] < 0 || s[q] >= ng || z[q] < 0 || z[q] >= ng || s[q] == z[q])
            return fail(MANTRA_E_INVALID, "pair %lld: (%d, %d) not two distinct nodes of graph %d", (long long)q,
                        s[q], z[q], gi);
    }
    if (node_f && (double)r * (double)g->n_total > 4e9) return fail(MANTRA_E_INVALID, "node_f too large");
    if (edge_f && (double)r * (double)g->m > 4e9) return fail(MANTRA_E_INVALID, "edge_f too large");
    std::lock_guard<std::mutex> lk(g->mu);
    hipSetDevice(g->device);
    g->last_ms = 0; g->last_launches = 0; g->last_W = 0; g->last_arcs = 0; g->last_tn = 0; g->last_te = 0;
    int32_t *dpg = nullptr, *dps = nullptr, *dpz = nullptr;
    void *drec = nullptr;
    double *dnf = nullptr, *def = nullptr;
    int rc = MANTRA_OK;
    auto cleanup = [&]() { hipFree(dpg); hipFree(dps); hipFree(dpz); hipFree(drec); hipFree(dnf); hipFree(def); };
    if (dalloc(&dps, (size_t)r) || dalloc(&dpz, (size_t)r) || dalloc((char **)&drec, (size_t)r * 24) ||
        (graph && dalloc(&dpg, (size_t)r)) || (node_f && dalloc(&dnf, (size_t)r * g->n_total)) ||
        (edge_f && dalloc(&def, (size_t)r * g->m))) {
        cleanup();
        (void)hipGetLastError();
        return fail(MANTRA_E_OOM, "count_pairs buffers");
    }
    {
        std::vector<int32_t> si((size_t)r), zi((size_t)r);
        for (int64_t q = 0; q < r; ++q) {
            int32_t b = g->seg_noff[graph ? graph[q] : 0];
            si[(size_t)q] = g->perm[(size_t)(b + s[q])] - b;
            zi[(size_t)q] = g->perm[(size_t)(b + z[q])] - b;
        }
        hipMemcpy(dps, si.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice);
        hipMemcpy(dpz, zi.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice);
    }
    if (graph) hipMemcpy(dpg, graph, sizeof(int32_t) * r, hipMemcpyHostToDevice);
    if (dnf) hipMemsetAsync(dnf, 0, sizeof(double) * r * g->n_total, g->st);
    if (def) hipMemsetAsync(def, 0, sizeof(double) * r * g->m, g->st);
    LaunchSpec sp;
    mantra_request rq;
    memset(&rq, 0, sizeof rq);
    rq.opt = opt; rq.t0 = t0; rq.t1 = t1;
    norm_window(rq);
    Acc none;
    DevReq d = make_req(rq, STREAM_PAIR, 0, 0, r, none, 0);
    d.Bsum = d.Wsum = d.Rsum = d.Esum = nullptr;
    sp.reqs.push_back(d);
    sp.npairs = r;
    sp.dpg = dpg; sp.dps = dps; sp.dpz = dpz; sp.drec = drec; sp.dnode_f = dnf; sp.dedge_f = def;
    u64 st[16];
    rc = run_sweep(g, sp, st);
    if (!rc) {
        if (hipMemcpy(out, drec, (size_t)r * 24, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(MANTRA_E_INTERNAL, "copy records");
        if (!rc && node_f) {
            std::vector<double> tmp((size_t)(r * g->n_total));
            if (hipMemcpy(tmp.data(), dnf, sizeof(double) * r * g->n_total, hipMemcpyDeviceToHost) != hipSuccess)
                rc = fail(MANTRA_E_INTERNAL, "copy node_f");
            else
                for (int64_t q = 0; q < r; ++q)
                    for (int64_t v = 0; v < g->n_total; ++v)
                        node_f[q * g->n_total + g->iperm[(size_t)v]] = tmp[(size_t)(q * g->n_total + v)];
        }
        if (!rc && edge_f) {
            std::vector<double> tmp((size_t)(r * g->m));
            if (hipMemcpy(tmp.data(), def, sizeof(double) * r * g->m, hipMemcpyDeviceToHost) != hipSuccess)
                rc = fail(MANTRA_E_INTERNAL, "copy edge_f");
            else
                for (int64_t q = 0; q < r; ++q)
                    for (int64_t i = 0; i < g->m_in; ++i)
                        edge_f[q * g->m_in + i] = tmp[(size_t)(q * g->m + g->in2k[(size_t)i])];
        }
    }
    cleanup();
    return rc;
}

int mantra_run(mantra_graph *g, const mantra_request *req, mantra_result *out) {
    if (!g || !req) return fail(MANTRA_E_INVALID, "graph or request is NULL");
    std::lock_guard<std::mutex> lk(g->mu);
    hipSetDevice(g->device);
    return run_request(g, *req, out);
}

int mantra_estimate(mantra_graph *g, mantra_opt opt, double eps, double delta, uint64_t seed, double *node_bc,
                    mantra_result *out) {
    mantra_request rq;
    memset(&rq, 0, sizeof rq);
    rq.opt = opt; rq.t0 = 0; rq.t1 = INT32_MAX; rq.eps = eps; rq.delta = delta; rq.seed = seed; rq.c = 25;
    rq.node_bc = node_bc;
    return mantra_run(g, &rq, out);
}

}  // extern "C"

// serving lives in mantra_serve.hip
