// Host runtime of the temporal-betweenness library: graph residency, the
// per-slab device state, launches of the sweep kernel and the progressive
// sampling driver of Algorithm 1 (blocking calls and the serving scheduler
// share the per-request state machine defined here).

#include <functional>

#include "mantra_int.h"

namespace mantra {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
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

// an input edge with its graph's local INPUT node ids (the stream is ordered
// by them, so that the order of a tick's edges is a function of the input)
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
            E[(size_t)i] = EdgeRec{gi, tt, v, u, i};
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
            const int32_t b = g->seg_noff[e.g];
            U.push_back(g->perm[(size_t)(b + e.u)] - b);
            V.push_back(g->perm[(size_t)(b + e.v)] - b);
            T.push_back(e.t);
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
    if (gm >= ((int64_t)1 << 31)) return fail(MANTRA_E_INVALID, "a tick holds %lld edges (at most 2^31-1)", (long long)gm);
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
    {
        // internal edge ids are below m < 2^32
        std::vector<uint32_t> ik((size_t)(g->m_in ? g->m_in : 1));
        for (int64_t i = 0; i < g->m_in; ++i) ik[(size_t)i] = (uint32_t)g->in2k[(size_t)i];
        HIPCHK(dalloc(&g->din2k, g->m_in));
        HIPCHK(hipMemcpy(g->din2k, ik.data(), sizeof(uint32_t) * ik.size(), hipMemcpyHostToDevice));
    }
    HIPCHK(dalloc(&g->dout, kOutChunk));
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
    HIPCHK(dalloc(&g->dstats, kStats));
    *out = g.release();
    return MANTRA_OK;
}

// ------------------------------------------------------------------ slabs

// A reached-set bitmap in LDS lets a batch skip the state loads of unreached
// tails; beyond 8 KB it costs more occupancy than it saves, and the bitmap
// is in the slab's global memory instead (in 16-byte words).
int lds_bitmap_ok(int64_t nmax) { return ((nmax + 31) / 32) * 4 <= 8 * 1024; }
size_t node_bytes_per_slab(int64_t nmax) { return lds_bitmap_ok(nmax) ? 0 : (size_t)((nmax + 127) / 128) * 16; }
// forward state of the top hub nodes in LDS
static int hub_nodes(const mantra_graph *g) { return (int)std::min<int64_t>(g->hub_nodes, g->nmax); }
size_t lds_bytes(const mantra_graph *g) {
    const int64_t nmax = g->nmax;
    size_t b = mantra_tab_lds_bytes();
    if (lds_bitmap_ok(nmax)) b += ((size_t)((nmax + 31) / 32) * 4 + 7) & ~(size_t)7;
    b += (size_t)hub_nodes(g) * 12;
    return b;
}

// device bytes of one slab's per-node state (F: 16 B, shared by the forward
// and the reverse; N: 8 B; touched: 4 B; the reached set's bit where the
// bitmap is not in LDS) and of its per-tick scratch (XS and AG: 16 B each per
// edge of the longest tick)
static size_t slab_state_bytes(const mantra_graph *g) {
    return (size_t)g->nmax * 28 + node_bytes_per_slab(g->nmax) + (size_t)g->gmax * 32 + 16;
}

// device memory and the share of it the slab pool (state and arc buffers)
// may take
static void device_mem(const mantra_graph *g, size_t *fr, size_t *tot) {
    *fr = 0;
    *tot = 0;
    hipSetDevice(g->device);
    hipMemGetInfo(fr, tot);
}
static size_t device_bytes(const mantra_graph *g) {
    size_t fr, tot;
    device_mem(g, &fr, &tot);
    return tot;
}
// Arc records (32 B each).  Each slab has a buffer of its own (own_cap
// arcs); a pair with more arcs takes chunks of kArcChunk arcs from a pool the
// launch shares, so that the arc room follows the pairs in flight rather
// than the largest pair times the grid.  The own buffer holds 2^18 arcs, or
// up to 2^20 where the resident grid's slabs with it still fit half of the
// pool's share of the device: pairs whose arcs run into the shared chunks
// are slower (on the 50k graph, 2^18 arcs cost the step about 10% against
// 6*10^5 or more, which only its longest pairs pass).
static const size_t kChunkBytes = (size_t)kArcChunk * 32;
static int resident_slabs(const mantra_graph *g);
static size_t slab_state_bytes(const mantra_graph *g);
static constexpr double kPoolShare = 0.75;
static int64_t own_cap(const mantra_graph *g) {
    if (g->user_cap > 0) return std::min<int64_t>(g->user_cap, g->m + 1);
    int64_t cap = (int64_t)1 << 18;
    const int64_t rs = resident_slabs(g);
    const size_t half = (size_t)(kPoolShare * (double)device_bytes(g)) / 2;
    const size_t st = slab_state_bytes(g);
    if (rs > 0 && half / (size_t)rs > st) {
        const int64_t fit = (int64_t)((half / (size_t)rs - st) / 33);
        cap = std::max<int64_t>(cap, std::min<int64_t>(fit, (int64_t)1 << 20));
    }
    return std::min<int64_t>(g->m + 1, cap);
}
// chunk-table entries per slab: enough for a pair with an arc per edge
static int64_t xmax_of(const mantra_graph *g, int64_t cap) {
    return cap >= g->m + 1 ? 0 : (g->m + 1 - cap + kArcChunk - 1) / kArcChunk;
}
static size_t slab_bytes(const mantra_graph *g, int64_t cap) {
    return slab_state_bytes(g) + (size_t)cap * 32 + (size_t)xmax_of(g, cap) * 4;
}
static size_t pool_bytes(const mantra_graph *g, const SlabPool &p) {
    return p.nslabs ? (size_t)p.nslabs * slab_bytes(g, p.cap) + (size_t)p.nchunks * kChunkBytes : 0;
}
// 75% of the device, less when other graphs or callers already hold memory
// (the graph's own pool counts as available).  The rest holds the graph,
// the per-request sums of served requests and the re-run pools.
static size_t pool_budget(const mantra_graph *g) {
    size_t fr, tot;
    device_mem(g, &fr, &tot);
    const size_t own = pool_bytes(g, g->pool);
    return (size_t)std::min(kPoolShare * (double)tot, 0.85 * (double)(fr + own));
}

// default device bytes the serving scheduler may give to per-request sums:
// what is free once the slab pool (the per-pair state and arc buffers every
// launch shares) holds its whole share of the device, less a margin for
// launch buffers and the multiword path
size_t serve_sums_budget(const mantra_graph *g) {
    size_t fr, tot;
    device_mem(g, &fr, &tot);
    const size_t own = pool_bytes(g, g->pool);
    const size_t share = (size_t)(kPoolShare * (double)tot);
    const size_t reserve = share > own ? share - own : 0;
    const size_t left = fr > reserve ? fr - reserve : 0;
    return std::max<size_t>((size_t)64 << 20, (size_t)(0.75 * (double)left));
}

// sweep workgroups the device holds at once (registers and LDS, as the
// runtime reports them)
static int resident_slabs(const mantra_graph *g) {
    hipDeviceProp_t pr;
    hipGetDeviceProperties(&pr, g->device);
    int cus = pr.multiProcessorCount > 0 ? pr.multiProcessorCount : 256;
    size_t lb = lds_bytes(g);
    int per_cu = mantra_sweep_occupancy(lb, lds_bitmap_ok(g->nmax) ? 0 : 1);
    if (per_cu <= 0) {
        int by_lds = (int)((160 * 1024) / (lb ? lb : 1));
        per_cu = std::min(8, std::max(1, by_lds));
    }
    return cus * per_cu;
}

// slabs whose state and own arc buffers fill half of the pool budget (large
// graphs); the other half holds the shared arc chunks
static int64_t slabs_by_memory(const mantra_graph *g) {
    return (int64_t)(pool_budget(g) / 2 / slab_bytes(g, own_cap(g)));
}

int auto_slabs(const mantra_graph *g) {
    if (g->user_slabs > 0) return g->user_slabs;
    return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)resident_slabs(g), slabs_by_memory(g)));
}

// shared chunks of a pool of ns slabs: the rest of the budget, no more than
// the slabs could ever hold
static int64_t auto_chunks(const mantra_graph *g, int ns, int64_t cap) {
    const int64_t xm = xmax_of(g, cap);
    if (xm == 0 || g->no_chunks) return 0;
    const size_t bud = pool_budget(g), slabs = (size_t)ns * slab_bytes(g, cap);
    const int64_t fit = bud > slabs ? (int64_t)((bud - slabs) / kChunkBytes) : 0;
    const int64_t n = std::min<int64_t>(fit, (int64_t)ns * xm);
    return g->max_chunks > 0 ? std::min<int64_t>(n, g->max_chunks) : n;
}

static int pool_ensure(mantra_graph *g, SlabPool &p, int nslabs, int64_t cap, int64_t nchunks) {
    int64_t nmax = g->nmax;
    int64_t gmax = g->gmax;
    if (p.nslabs >= nslabs && p.cap == cap && p.nmax == nmax && p.gmax >= gmax && p.nchunks >= nchunks)
        return MANTRA_OK;
    p.release();
    p.nmax = nmax; p.cap = cap; p.gmax = gmax;
    size_t ns = (size_t)nslabs;
    const int64_t xm = xmax_of(g, cap), xwords = (nchunks + 31) / 32;
    // Allocation order: the shared chunks and the arc buffers first, the
    // per-node state that the sweep gathers from last.  Measured on the 2M-node
    // graph (fresh processes, 1,280 slabs): 4,846-4,882 ms per launch of 8,192
    // sfm pairs this way against 5,272-5,372 ms with the per-node state
    // allocated first.  The cause is not established: the arrays get other
    // device addresses, and the state-first pool reallocated after a larger
    // pool was freed ran 6-8% faster too.
    if ((nchunks > 0 && (dalloc(&p.xarcs, (size_t)nchunks * 4 * (size_t)kArcChunk) ||
                         dalloc(&p.xfree, (size_t)xwords) || dalloc(&p.xtab, ns * (size_t)xm))) ||
        (node_bytes_per_slab(nmax) && dalloc(&p.BM, ns * node_bytes_per_slab(nmax))) || dalloc(&p.hdr, ns * 4) ||
        dalloc(&p.XS, ns * (size_t)gmax * 2) || dalloc(&p.arcs, ns * (size_t)cap * 4) ||
        dalloc(&p.touched, ns * nmax) || dalloc(&p.AG, ns * (size_t)gmax * 2) ||
        dalloc(&p.N, ns * nmax) || dalloc(&p.F, ns * nmax * 2)) {
        p.release();
        (void)hipGetLastError();
        return fail(MANTRA_E_OOM, "slab pool: %d slabs x (%lld nodes, %lld arcs) + %lld arc chunks does not fit",
                    nslabs, (long long)nmax, (long long)cap, (long long)nchunks);
    }
    p.nchunks = nchunks;
    p.xmax = nchunks > 0 ? xm : 0;
    if (nchunks > 0) {
        // every chunk free
        std::vector<u32> bits((size_t)xwords, ~0u);
        if (nchunks % 32) bits.back() = (1u << (nchunks % 32)) - 1u;
        HIPCHK(hipMemcpy(p.xfree, bits.data(), sizeof(u32) * (size_t)xwords, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemsetAsync(p.F, 0, sizeof(u64) * ns * nmax * 2, g->st));
    HIPCHK(hipMemsetAsync(p.N, 0, sizeof(u64) * ns * nmax, g->st));
    HIPCHK(hipMemsetAsync(p.hdr, 0, sizeof(u32) * ns * 4, g->st));
    if (p.BM) HIPCHK(hipMemsetAsync(p.BM, 0, ns * node_bytes_per_slab(nmax), g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    p.nslabs = nslabs;
    return MANTRA_OK;
}

// the RTB kernel's per-node first arrivals (16 B per node per slab), on first use
static int pool_need_T(mantra_graph *g, SlabPool &p) {
    if (p.T || !p.nslabs) return MANTRA_OK;
    if (dalloc(&p.T, (size_t)p.nslabs * (size_t)p.nmax * 2)) {
        (void)hipGetLastError();
        return fail(MANTRA_E_OOM, "RTB state of %d slabs x %lld nodes", p.nslabs, (long long)p.nmax);
    }
    return MANTRA_OK;
}

// the multiword path's slabs: per node the forward and reverse state, N and
// the touched list; per edge of the longest tick its scratch; arcs for every
// edge of the graph (a pair's arcs never outnumber its window)
static size_t wide_slab_bytes(const mantra_graph *g, int64_t cap) {
    return (size_t)g->nmax * (16 + 24 * kWide + 4) + (size_t)g->gmax * (4 + 8 * kWide) +
           (size_t)cap * 8 * (3 + kWide) + 16;
}
static int wide_ensure(mantra_graph *g, int nslabs, int64_t cap) {
    WidePool &p = g->wide;
    if (p.nslabs >= nslabs && p.cap >= cap && p.nmax == g->nmax && p.gmax >= g->gmax) return MANTRA_OK;
    p.release();
    const size_t ns = (size_t)nslabs, n = (size_t)g->nmax, gm = (size_t)g->gmax;
    if (dalloc(&p.ST, ns * n) || dalloc(&p.SS, ns * n * kWide) || dalloc(&p.RT, ns * n) ||
        dalloc(&p.RA, ns * n * kWide) || dalloc(&p.NV, ns * n * kWide) || dalloc(&p.touched, ns * n) ||
        dalloc(&p.TL, ns * gm) || dalloc(&p.TC, ns * gm * kWide) || dalloc(&p.AR, ns * (size_t)cap * (3 + kWide)) ||
        dalloc(&p.hdr, ns * 4)) {
        p.release();
        (void)hipGetLastError();
        return fail(MANTRA_E_OOM, "multiword path: %d slabs x %lld nodes", nslabs, (long long)n);
    }
    HIPCHK(hipMemsetAsync(p.ST, 0, sizeof(u64) * ns * n, g->st));
    HIPCHK(hipMemsetAsync(p.RT, 0, sizeof(u64) * ns * n, g->st));
    HIPCHK(hipMemsetAsync(p.NV, 0, sizeof(u64) * ns * n * kWide, g->st));
    HIPCHK(hipMemsetAsync(p.hdr, 0, sizeof(u32) * ns * 4, g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    p.nslabs = nslabs;
    p.nmax = g->nmax;
    p.gmax = g->gmax;
    p.cap = cap;
    return MANTRA_OK;
}

// whether device memory, not residency, bounds the automatic grid (large
// graphs)
static bool memory_bound(const mantra_graph *g) { return slabs_by_memory(g) < (int64_t)resident_slabs(g); }

// The pool a launch of ns slabs runs on.  Where residency bounds the grid,
// a pool with at least ns slabs (and the same own arc room) is kept, so that
// alternating grids (the autotuner's) do not reallocate it.  Where memory
// bounds it, the pool is sized for this grid: slabs and their own buffers,
// and the shared chunks in the rest of the budget.
static int pool_for(mantra_graph *g, int ns) {
    const int64_t cap = own_cap(g);
    SlabPool &p = g->pool;
    if (p.nslabs >= ns && p.cap == cap && p.nmax == g->nmax && p.gmax >= g->gmax &&
        (p.nchunks == 0) == (auto_chunks(g, ns, cap) == 0) && (!memory_bound(g) || p.nslabs == ns))
        return MANTRA_OK;
    if (p.nslabs) p.release();
    return pool_ensure(g, p, ns, cap, auto_chunks(g, ns, cap));
}

// Slab state words carry their pair's tag (the slab's pair serial, +2 per
// pair), a u32 that a slab carries across launches.  Before it could wrap --
// a word left by a pair 2^31 pairs earlier would then read as current -- the
// pool's tagged words and serials are cleared and the slabs start over.  The
// kernels report each slab's serial; a launch advances it by at most 2 per
// pair it holds.
static constexpr u64 kStampLimit = 1ull << 31;
static int stamps_clear(mantra_graph *g, SlabPool &p) {
    const size_t ns = (size_t)p.nslabs;
    HIPCHK(hipMemsetAsync(p.F, 0, sizeof(u64) * ns * (size_t)p.nmax * 2, g->st));
    HIPCHK(hipMemsetAsync(p.hdr, 0, sizeof(u32) * ns * 4, g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    p.serial_hi = 0;
    return MANTRA_OK;
}
static int stamps_before(mantra_graph *g, SlabPool &p, int64_t slots) {
    if (p.serial_hi + 2 * (u64)(slots + 1) >= 2 * kStampLimit) return stamps_clear(g, p);
    return MANTRA_OK;
}
static int stamps_after(mantra_graph *g, SlabPool &p, const u64 *st) {
    p.serial_hi = std::max(p.serial_hi, st[12]);
    if (p.serial_hi >= kStampLimit) return stamps_clear(g, p);
    return MANTRA_OK;
}
static int wide_stamps(mantra_graph *g, int64_t slots, const u64 *st) {
    WidePool &p = g->wide;
    if (st) p.serial_hi = std::max(p.serial_hi, st[12]);
    const bool before = !st && p.serial_hi + 2 * (u64)(slots + 1) >= 2 * kStampLimit;
    if (!before && p.serial_hi < kStampLimit) return MANTRA_OK;
    const size_t ns = (size_t)p.nslabs, n = (size_t)p.nmax;
    HIPCHK(hipMemsetAsync(p.ST, 0, sizeof(u64) * ns * n, g->st));
    HIPCHK(hipMemsetAsync(p.RT, 0, sizeof(u64) * ns * n, g->st));
    HIPCHK(hipMemsetAsync(p.hdr, 0, sizeof(u32) * ns * 4, g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    p.serial_hi = 0;
    return MANTRA_OK;
}

template <class T>
static int grow(T **p, int64_t &cap, int64_t need, int64_t minimum) {
    if (need <= cap && *p) return MANTRA_OK;
    hipFree(*p);
    *p = nullptr;
    cap = std::max(need, minimum);
    HIPCHK(dalloc(p, (size_t)cap));
    return MANTRA_OK;
}

void RoundGraph::release() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    ns = 0;
}

// the kernels of one launch: clear the counters, order the slots (longest
// estimated window first), sweep; with rg, also the request's reduction
static hipError_t launch_sweep(const LaunchArgs &a, int mode, int ns, size_t lb, hipStream_t st) {
    if (mode == MODE_DISTANCES) return mantra_launch_sweep_sources(&a, ns, lb, st);
    if (mode == MODE_TRK) return mantra_launch_sweep_trk(&a, ns, lb, st);
    if (mode == MODE_RTB) return mantra_launch_sweep_rtb(&a, ns, lb, st);
    return mantra_launch_sweep(&a, ns, lb, st);
}

static int issue_kernels(mantra_graph *g, LaunchArgs &a, int ns, size_t lb, const RoundGraph *rg, int mode) {
    HIPCHK(mantra_launch_clear(g->dwork, (u32 *)g->dretry, (u32 *)g->dwide, g->dstats, g->st));
    if (g->order_mode == MANTRA_ORDER_LONGEST_FIRST && a.npairs > ns) {
        HIPCHK(mantra_launch_order(&a, g->dbucket, g->dhist, g->dorder, g->st));
        a.pq = g->dorder;
    }
    if (!rg) HIPCHK(hipEventRecord(g->ev0, g->st));
    HIPCHK(launch_sweep(a, mode, ns, lb, g->st));
    if (!rg) HIPCHK(hipEventRecord(g->ev1, g->st));
    if (rg) {
        ReduceArgs ra;
        ra.W = rg->W; ra.B = rg->B; ra.R = rg->R; ra.n = g->n_total; ra.c = rg->c; ra.part = g->dpart;
        HIPCHK(mantra_launch_reduce(&ra, reduce_blocks(g->n_total), g->st));
    }
    return MANTRA_OK;
}

// launch the sweep over all pairs of spec; re-run pairs whose arcs did not
// fit with a pool of few slabs and the largest capacity.  With rg (a
// progressive round of one blocking request), the launch sequence and the
// request's reduction are one HIP graph, captured for rg->cap slots on first
// use and replayed with the slice and its pair count in device memory.
int run_sweep(mantra_graph *g, const LaunchSpec &sp, SweepOut &o, RoundGraph *rg) {
    memset(o.st, 0, sizeof o.st);
    o.ms = 0;
    o.first_ms = 0;
    o.launches = 0;
    o.reduced = false;
    if (sp.npairs <= 0) return MANTRA_OK;
    hipSetDevice(g->device);
    const int64_t slots = rg ? std::max(rg->cap, sp.npairs) : sp.npairs;
    int ns = auto_slabs(g);
    if ((int64_t)ns > slots) ns = (int)slots;
    if (g->per_pair) ns = 1;
    // the pool is sized for the graph's grid (a smaller launch uses part of it)
    int rc = pool_for(g, auto_slabs(g));
    if (rc) return rc;
    if ((rc = stamps_before(g, g->pool, slots))) return rc;
    if (sp.mode == MODE_RTB && (rc = pool_need_T(g, g->pool))) return rc;
    int64_t rcap = g->dreq_cap;
    if ((rc = grow(&g->dreqs, rcap, (int64_t)sp.reqs.size(), 64))) return rc;
    g->dreq_cap = (int)rcap;
    if ((rc = grow(&g->dretry, g->retry_cap, slots + 1, 4096))) return rc;
    if ((rc = grow(&g->dwide, g->wide_cap, slots + 1, 4096))) return rc;
    int64_t oc = g->order_cap;
    if ((rc = grow(&g->dbucket, oc, slots, 4096))) return rc;
    if ((rc = grow(&g->dorder, g->order_cap, slots, 4096))) return rc;
    if (!g->dhist) HIPCHK(dalloc(&g->dhist, (size_t)kOrderBuckets));
    if (!g->dnp) HIPCHK(dalloc(&g->dnp, 1));
    if (rg && (rc = reduce_part_ensure(g, rg->c))) return rc;
    HIPCHK(hipMemcpyAsync(g->dreqs, sp.reqs.data(), sizeof(DevReq) * sp.reqs.size(), hipMemcpyHostToDevice, g->st));
    LaunchArgs a;
    memset(&a, 0, sizeof a);
    a.g = g->dev();
    a.sl = g->pool.view();
    a.reqs = g->dreqs;
    a.nreq = (int32_t)sp.reqs.size();
    a.lds_bitmap = lds_bitmap_ok(g->nmax);
    a.hub_nodes = hub_nodes(g);
    a.npairs = slots;
    a.npairs_dev = nullptr;
    a.qbase = 0;
    a.pg = sp.dpg; a.ps = sp.dps; a.pz = sp.dpz; a.pq = nullptr;
    a.rec = sp.drec;
    a.node_f = sp.dnode_f;
    a.edge_f = sp.dedge_f;
    a.work = g->dwork;
    a.stats = g->dstats;
    a.retry = g->dretry;
    a.wide = (sp.mode == MODE_PAIRS && g->wide_mode != MANTRA_WIDE_NONE) ? g->dwide : nullptr;  // saturated pairs:
    a.wide_fm = g->wide_mode == MANTRA_WIDE_ALL ? 1 : 0;                                        // the multiword path
    const size_t lb = lds_bytes(g);
    float ms = 0;
    if (g->per_pair) {
        // the unbatched form: one single-workgroup launch per pair
        HIPCHK(mantra_launch_clear(g->dwork, (u32 *)g->dretry, (u32 *)g->dwide, g->dstats, g->st));
        HIPCHK(hipEventRecord(g->ev0, g->st));
        for (int64_t q = 0; q < sp.npairs; ++q) {
            a.qbase = q;
            a.npairs = q + 1;
            HIPCHK(hipMemsetAsync(g->dwork, 0, sizeof(u32), g->st));
            HIPCHK(launch_sweep(a, sp.mode, 1, lb, g->st));
            o.launches += 1;
        }
        HIPCHK(hipEventRecord(g->ev1, g->st));
        a.qbase = 0;
        a.npairs = sp.npairs;
    } else if (rg) {
        HIPCHK(hipMemcpyAsync(g->dnp, &sp.npairs, sizeof(int64_t), hipMemcpyHostToDevice, g->st));
        a.npairs_dev = g->dnp;
        // buffers moved since the capture: capture again
        if (rg->exec && (rg->ns != ns || memcmp(&rg->args, &a, sizeof a) != 0)) rg->release();
        if (!rg->exec) {
            rg->cap = slots;
            rg->ns = ns;
            memcpy(&rg->args, &a, sizeof a);
            HIPCHK(hipStreamBeginCapture(g->st, hipStreamCaptureModeThreadLocal));
            int crc = issue_kernels(g, a, ns, lb, rg, sp.mode);
            hipGraph_t gr = nullptr;
            hipError_t e = hipStreamEndCapture(g->st, &gr);
            if (crc) { if (gr) hipGraphDestroy(gr); return crc; }
            HIPCHK(e);
            rg->graph = gr;
            HIPCHK(hipGraphInstantiate(&rg->exec, rg->graph, nullptr, nullptr, 0));
        }
        HIPCHK(hipEventRecord(g->ev0, g->st));
        HIPCHK(hipGraphLaunch(rg->exec, g->st));
        HIPCHK(hipEventRecord(g->ev1, g->st));
        o.launches += 1;
        o.reduced = true;
    } else {
        if ((rc = issue_kernels(g, a, ns, lb, nullptr, sp.mode))) return rc;
        o.launches += 1;
    }
    int32_t nretry = 0;
    HIPCHK(hipMemcpyAsync(&nretry, g->dretry, sizeof(int32_t), hipMemcpyDeviceToHost, g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
    o.ms += ms;
    o.first_ms = ms;
    u64 st1[kStats];
    HIPCHK(hipMemcpy(st1, g->dstats, sizeof(u64) * kStats, hipMemcpyDeviceToHost));
    if ((rc = stamps_after(g, g->pool, st1))) return rc;
    if (nretry > 0 && g->pool.nchunks > 0 && !g->per_pair) {
        // pairs that found no free shared chunk run again on the same pool,
        // alone: every chunk is free again, and they are few
        o.reduced = false;
        std::vector<int32_t> q((size_t)nretry + 1);
        HIPCHK(hipMemcpy(q.data(), g->dretry, sizeof(int32_t) * (nretry + 1), hipMemcpyDeviceToHost));
        int32_t *dq = nullptr;
        HIPCHK(dalloc(&dq, (size_t)nretry));
        HIPCHK(hipMemcpy(dq, q.data() + 1, sizeof(int32_t) * nretry, hipMemcpyHostToDevice));
        if ((rc = stamps_before(g, g->pool, nretry))) { hipFree(dq); return rc; }
        HIPCHK(mantra_launch_clear(g->dwork, (u32 *)g->dretry, nullptr, g->dstats, g->st));  // keeps the
        a.sl = g->pool.view();                                                                  // multiword list
        a.npairs = nretry;
        a.npairs_dev = nullptr;
        a.qbase = 0;
        a.pq = dq;
        const int nsr = (int)std::min<int64_t>(std::min<int64_t>(nretry, g->pool.nslabs), g->pool.nchunks);
        HIPCHK(hipEventRecord(g->ev0, g->st));
        HIPCHK(launch_sweep(a, sp.mode, nsr, lb, g->st));
        HIPCHK(hipEventRecord(g->ev1, g->st));
        HIPCHK(hipStreamSynchronize(g->st));
        HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
        o.ms += ms;
        o.launches += 1;
        u64 st2[kStats];
        HIPCHK(hipMemcpy(st2, g->dstats, sizeof(u64) * kStats, hipMemcpyDeviceToHost));
        if ((rc = stamps_after(g, g->pool, st2))) { hipFree(dq); return rc; }
        for (int i = 0; i < 16; ++i)
            if ((i != 5 && i < 9) || (i >= 14 && i < 18)) st1[i] += st2[i];
        // the ones still without room (the list holds their original slots)
        // go to the next stage
        int32_t n2 = 0;
        HIPCHK(hipMemcpy(&n2, g->dretry, sizeof(int32_t), hipMemcpyDeviceToHost));
        hipFree(dq);
        nretry = n2;
    }
    if (nretry > 0) {
        // pairs whose arcs overflowed get slabs that hold every edge of the
        // graph, as many as a fifth of device memory allows
        o.reduced = false;
        int64_t cap2 = g->m + 1;
        size_t fr, tot;
        device_mem(g, &fr, &tot);
        int64_t fit = (int64_t)(std::min(tot / 5, fr / 2) / (slab_state_bytes(g) + (size_t)cap2 * 32));
        int ns2 = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int>(nretry, 64), fit));
        rc = pool_ensure(g, g->pool_big, ns2, cap2, 0);
        if (rc) return rc;
        if (sp.mode == MODE_RTB && (rc = pool_need_T(g, g->pool_big))) return rc;
        std::vector<int32_t> q((size_t)nretry + 1);
        HIPCHK(hipMemcpy(q.data(), g->dretry, sizeof(int32_t) * (nretry + 1), hipMemcpyDeviceToHost));
        int32_t *dq = nullptr;
        HIPCHK(dalloc(&dq, (size_t)nretry));
        HIPCHK(hipMemcpy(dq, q.data() + 1, sizeof(int32_t) * nretry, hipMemcpyHostToDevice));
        HIPCHK(mantra_launch_clear(g->dwork, (u32 *)g->dretry, nullptr, g->dstats, g->st));  // keeps the
        a.sl = g->pool_big.view();                                                              // multiword list
        a.npairs = nretry;
        a.npairs_dev = nullptr;
        a.qbase = 0;
        a.pq = dq;
        HIPCHK(hipEventRecord(g->ev0, g->st));
        HIPCHK(launch_sweep(a, sp.mode, ns2, lb, g->st));
        HIPCHK(hipEventRecord(g->ev1, g->st));
        HIPCHK(hipStreamSynchronize(g->st));
        HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
        o.ms += ms;
        o.launches += 1;
        u64 st2[kStats];
        HIPCHK(hipMemcpy(st2, g->dstats, sizeof(u64) * kStats, hipMemcpyDeviceToHost));
        hipFree(dq);
        g->pool_big.release();  // rare and large: not kept between launches
        int32_t n2 = 0;
        HIPCHK(hipMemcpy(&n2, g->dretry, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (n2 > 0) return fail(MANTRA_E_INTERNAL, "arc buffer of a full window overflowed");
        for (int i = 0; i < 16; ++i)
            if ((i != 5 && i < 9) || (i >= 14 && i < 18)) st1[i] += st2[i];
    }
    int32_t nwide = 0;
    if (a.wide) HIPCHK(hipMemcpy(&nwide, g->dwide, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (nwide > 0) {
        // pairs whose 64-bit counts saturated: exact multiword counts, one
        // lane per pair, as many slabs as an eighth of device memory holds
        o.reduced = false;
        const int64_t cap3 = g->m + 1;
        size_t fr, tot;
        device_mem(g, &fr, &tot);
        const int64_t fit = (int64_t)(std::min(tot / 8, fr / 2) / wide_slab_bytes(g, cap3));
        const int ns3 = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int>(nwide, 128), fit));
        if ((rc = wide_ensure(g, std::max(ns3, g->wide.nslabs), cap3))) return rc;
        if ((rc = wide_stamps(g, nwide, nullptr))) return rc;
        HIPCHK(mantra_launch_clear(g->dwork, (u32 *)g->dretry, nullptr, g->dstats, g->st));
        a.npairs = nwide;
        a.npairs_dev = nullptr;
        a.qbase = 0;
        a.pq = g->dwide + 1;
        const WideSlabs wv = g->wide.view();
        HIPCHK(hipEventRecord(g->ev0, g->st));
        HIPCHK(mantra_launch_wide(&a, &wv, ns3, g->st));
        HIPCHK(hipEventRecord(g->ev1, g->st));
        HIPCHK(hipStreamSynchronize(g->st));
        HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
        o.ms += ms;
        o.launches += 1;
        u64 st3[kStats];
        HIPCHK(hipMemcpy(st3, g->dstats, sizeof(u64) * kStats, hipMemcpyDeviceToHost));
        if ((rc = wide_stamps(g, nwide, st3))) return rc;
        st1[2] += st3[2];
        st1[4] += st3[4];
        st1[6] += st3[6];
    }
    memcpy(o.st, st1, sizeof(st1));
    // busy share of the first launch's persistent grid
    const u64 span = st1[10] - ~st1[11];
    o.balance = span && !g->per_pair ? (double)st1[9] / ((double)ns * (double)span) : 1.0;
    if (st1[6]) return fail(MANTRA_E_INTERNAL, "%llu pairs failed flow conservation", (unsigned long long)st1[6]);
    return MANTRA_OK;
}

// blocking calls report their work through mantra_last_timing
void timing_reset(mantra_graph *g) {
    g->last_ms = 0; g->last_launches = 0; g->last_W = 0; g->last_arcs = 0; g->last_tn = 0; g->last_te = 0;
    g->last_live = 0; g->last_dead = 0; g->last_fwd_ticks = 0; g->last_rev_ticks = 0;
    g->last_busy_ms = 0;
}
void timing_add(mantra_graph *g, const SweepOut &o) {
    g->last_busy_ms += o.balance * o.ms;
    g->last_ms += o.ms;
    g->last_launches += o.launches;
    g->last_W += (int64_t)o.st[0];
    g->last_arcs += (int64_t)o.st[1];
    g->last_tn += (int64_t)o.st[7];
    g->last_te += (int64_t)o.st[8];
    g->last_live += (int64_t)o.st[14];
    g->last_dead += (int64_t)o.st[15];
    g->last_fwd_ticks += (int64_t)o.st[16];
    g->last_rev_ticks += (int64_t)o.st[17];
}

// per-block partials of max W, sum B, max R_j
int reduce_blocks(int64_t n) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256)); }

int reduce_part_ensure(mantra_graph *g, int c) {
    if (g->dpart && g->part_c >= c) return MANTRA_OK;
    hipFree(g->dpart);
    g->dpart = nullptr;
    g->part_blocks = 1024;
    g->part_c = std::max(c, 64);
    HIPCHK(dalloc(&g->dpart, (size_t)1024 * (2 + g->part_c)));
    return MANTRA_OK;
}

// launch (unless a graph replay already did) and read back the reduction
static int reduce(mantra_graph *g, const double *W, const double *B, const double *R, int64_t n, int c,
                  double *maxW, double *sumB, std::vector<double> &maxR, bool launched = false) {
    const int blocks = reduce_blocks(n);
    int rc = reduce_part_ensure(g, c);
    if (rc) return rc;
    if (!launched) {
        ReduceArgs ra;
        ra.W = W; ra.B = B; ra.R = R; ra.n = n; ra.c = c; ra.part = g->dpart;
        HIPCHK(mantra_launch_reduce(&ra, blocks, g->st));
    }
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

// a slice of count pairs of one request's stream.  Launch slot q of the slice
// takes stream index base + (q - qoff); for graph = -1 (fixed samples over
// packed graphs) that index i names graph i / per_graph and its pair
// i % per_graph.
static DevReq make_req(const mantra_request &rq, int stream, int64_t base, int64_t qoff, int64_t count,
                       const Acc *acc, int c) {
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
    d.mode = (rq.flags & MANTRA_F_RTB) ? MODE_RTB : (rq.flags & MANTRA_F_TRK) ? MODE_TRK : MODE_PAIRS;
    if (acc) {
        d.Bsum = acc->B;
        d.Wsum = acc->W;
        d.Rsum = c > 0 ? acc->R : nullptr;
        d.Esum = acc->E;
    }
    return d;
}

int check_request(const mantra_graph *g, const mantra_request &rq) {
    if (rq.opt < MANTRA_SH || rq.opt > MANTRA_PFM) return fail(MANTRA_E_INVALID, "unknown optimality %d", (int)rq.opt);
    if (!rq.node_bc) return fail(MANTRA_E_INVALID, "node_bc is NULL");
    int c = rq.c ? rq.c : 25;
    if (c < 1 || c > 64) return fail(MANTRA_E_INVALID, "c = %d outside 1..64", c);
    if ((rq.flags & MANTRA_F_TRK) && (rq.flags & MANTRA_F_RTB))
        return fail(MANTRA_E_INVALID, "MANTRA_F_TRK and MANTRA_F_RTB are two estimators: pick one");
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

// Outputs in the caller's order: rows of `nin` values (input node or edge
// order), value i of row q being src[q * nsrc + idx[i]] / r, the value of the
// internal node or edge that input id i became, divided by the sample size
// (r = 0: the value itself).  This launch writes the flattened outputs
// o .. o + len - 1 to dst[0 .. len - 1], one thread per output.
template <typename I>
__global__ void __launch_bounds__(256) k_out(const double *src, const I *idx, int64_t nin, int64_t nsrc, int64_t o,
                                             int64_t len, double r, double *dst) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) {
        const int64_t j = o + i;
        const int64_t q = j < nin ? 0 : j / nin;
        const double x = src[q * nsrc + idx[j - q * nin]];
        dst[i] = r > 0 ? x / r : x;
    }
}

// host[q * nin + i] = src[q * nsrc + idx[i]] / r for rows q < rows, written on
// the device in the caller's order and copied out a piece at a time through
// the graph's staging buffer (callers hold the graph's lock)
template <typename I>
static int copy_out(mantra_graph *g, double *host, const double *src, const I *idx, int64_t nin, int64_t nsrc,
                    int64_t rows, double r) {
    const int64_t n = nin * rows;
    for (int64_t o = 0; o < n; o += kOutChunk) {
        const int64_t len = std::min(kOutChunk, n - o);
        const int blocks = (int)std::min<int64_t>((len + 255) / 256, 8192);
        hipLaunchKernelGGL(k_out<I>, dim3(blocks), dim3(256), 0, g->st, src, idx, nin, nsrc, o, len, r, g->dout);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(host + o, g->dout, sizeof(double) * len, hipMemcpyDeviceToHost, g->st));
    }
    return MANTRA_OK;
}

static int finish_outputs(mantra_graph *g, const mantra_request &rq, Acc &acc, int64_t r) {
    if (r <= 0) {
        std::fill(rq.node_bc, rq.node_bc + g->n_total, 0.0);
        if (rq.edge_bc && acc.E) std::fill(rq.edge_bc, rq.edge_bc + g->m_in, 0.0);
        return MANTRA_OK;
    }
    int rc = copy_out(g, rq.node_bc, acc.B, g->dperm, g->n_total, g->n_total, 1, (double)r);
    if (!rc && rq.edge_bc && acc.E) rc = copy_out(g, rq.edge_bc, acc.E, g->din2k, g->m_in, g->m, 1, (double)r);
    HIPCHK(hipStreamSynchronize(g->st));
    return rc;
}

size_t req_mem_bytes(const mantra_graph *g, const mantra_request &rq) {
    const int c = rq.c ? rq.c : 25;
    const bool edges = (rq.flags & MANTRA_F_EDGE_BC) && rq.edge_bc;
    size_t b = sizeof(double) * (size_t)g->n_total * (size_t)(2 + c);
    if (edges) b += sizeof(double) * (size_t)g->m;
    if (rq.fixed_r <= 0) b += sizeof(double) * (size_t)g->n_total * 3;  // bootstrap sums
    return b + sizeof(u64) * RS_N;
}

void req_release(ReqRun &q) {
    q.rg.release();
    q.acc.release();
    q.boot.release();
    hipFree(q.rstat);
    q.rstat = nullptr;
}

static int rstat_zero(mantra_graph *g, ReqRun &q) {
    HIPCHK(hipMemsetAsync(q.rstat, 0, sizeof(u64) * RS_N, g->st));
    return MANTRA_OK;
}

int req_begin(mantra_graph *g, ReqRun &q) {
    if (q.t_start == std::chrono::steady_clock::time_point()) q.t_start = std::chrono::steady_clock::now();
    memset(&q.R, 0, sizeof q.R);
    int rc = check_request(g, q.rq);
    if (rc) return rc;
    norm_window(q.rq);
    q.c = q.rq.c ? q.rq.c : 25;
    q.edges = (q.rq.flags & MANTRA_F_EDGE_BC) && q.rq.edge_bc;
    if (q.rq.opt == MANTRA_FM) q.R.flags |= MANTRA_RES_NO_GUARANTEE;
    q.mem_bytes = req_mem_bytes(g, q.rq);
    hipSetDevice(g->device);
    HIPCHK(dalloc(&q.rstat, RS_N));
    if ((rc = rstat_zero(g, q))) return rc;
    if ((rc = acc_alloc(g, q.acc, q.c, q.edges))) return rc;
    if ((rc = acc_zero(g, q.acc))) return rc;
    q.prev = 0;
    q.issued = 0;
    q.round = 0;
    if (q.rq.fixed_r > 0) {
        q.phase = ReqRun::ROUND;
        q.target = q.rq.fixed_r * g->G;
        return MANTRA_OK;
    }
    // bootstrap: s' pairs of their own stream, at delta/2 of the budget
    q.phase = ReqRun::BOOT;
    q.R.s_boot = bnd::boot(q.rq.eps, q.rq.delta);
    q.target = q.R.s_boot;
    if ((rc = acc_alloc(g, q.boot, 0, false))) return rc;
    return acc_zero(g, q.boot);
}

DevReq req_slice(ReqRun &q, int64_t count, int64_t qoff) {
    DevReq d;
    const int64_t base = q.prev + q.issued;
    if (q.phase == ReqRun::BOOT) {
        d = make_req(q.rq, STREAM_BOOT, base, qoff, count, &q.boot, 0);
    } else {
        d = make_req(q.rq, STREAM_PAIR, base, qoff, count, &q.acc, q.c);
        if (q.rq.fixed_r > 0) {
            // fixed samples: fixed_r pairs of each graph, graph-major
            d.graph = -1;
            d.per_graph = q.rq.fixed_r;
        }
    }
    d.rstat = q.rstat;
    q.issued += count;
    return d;
}

// counters of the finished phase
static int phase_stats(mantra_graph *g, ReqRun &q, u64 rs[RS_N]) {
    HIPCHK(hipMemcpyAsync(rs, q.rstat, sizeof(u64) * RS_N, hipMemcpyDeviceToHost, g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    int rc = rstat_zero(g, q);
    if (rc) return rc;
    q.R.window_edges += (int64_t)rs[RS_WINDOW];
    q.R.arcs += (int64_t)rs[RS_ARCS];
    if (rs[RS_HOPS]) return fail(MANTRA_E_LIMIT, "a hop count exceeded 65534");
    return MANTRA_OK;
}

int req_advance(mantra_graph *g, ReqRun &q) {
    if (q.phase == ReqRun::DONE || q.issued < q.target - q.prev) return MANTRA_OK;
    u64 rs[RS_N];
    int rc = phase_stats(g, q, rs);
    if (rc) return rc;
    const int c = q.c;
    // a sampled pair whose counts saturated voids the request's estimates
    // (MANTRA_E_OVERFLOW, never rounded): it stops at the end of that phase
    // instead of running the rest of its schedule for nothing
    if (rs[RS_OVERFLOW]) {
        q.R.n_overflow += (int64_t)rs[RS_OVERFLOW];
        q.R.n_reachable += q.phase == ReqRun::BOOT ? 0 : (int64_t)rs[RS_REACHABLE];
        if (q.phase == ReqRun::ROUND) {
            q.round += 1;
            q.R.rounds = q.round;
            q.R.samples = q.rq.fixed_r > 0 ? q.rq.fixed_r : q.target;
        }
        q.phase = ReqRun::DONE;
        return MANTRA_OK;
    }
    if (q.phase == ReqRun::BOOT) {
        double mw = 0, sumb = 0;
        std::vector<double> mr;
        if ((rc = reduce(g, q.boot.W, q.boot.B, q.boot.R, g->n_total, 0, &mw, &sumb, mr))) return rc;
        q.boot.release();
        const int64_t sb = q.R.s_boot;
        q.R.rho_hat = sumb / (double)sb;
        q.R.v_hat = std::min(0.25, std::max(mw, 0.0) / (double)sb);
        int64_t om = std::max<int64_t>(sb, bnd::omega(q.R.v_hat, q.R.rho_hat, q.rq.eps, q.rq.delta / 2.0, g->n_total));
        if (q.rq.max_samples > 0) om = std::min(om, q.rq.max_samples);
        int64_t s1 = q.rq.s1 > 0 ? q.rq.s1 : bnd::first(sb, om, q.R.v_hat, q.rq.eps, q.rq.delta / 4.0);
        s1 = std::min(s1, om);
        q.om = om;
        q.R.omega = om;
        q.R.s1 = s1;
        q.phase = ReqRun::ROUND;
        q.prev = 0;
        q.issued = 0;
        q.target = s1;
        return MANTRA_OK;
    }
    // a round (or the fixed sample) is complete
    q.R.n_reachable += (int64_t)rs[RS_REACHABLE];
    q.round += 1;
    const int64_t r = q.rq.fixed_r > 0 ? q.rq.fixed_r : q.target;
    q.R.rounds = q.round;
    q.R.samples = r;
    if (g->G == 1) {
        double mw, sumB;
        std::vector<double> mr;
        if ((rc = reduce(g, q.acc.W, q.acc.B, q.acc.R, g->n_total, c, &mw, &sumB, mr, q.reduced))) return rc;
        const double W = std::max(mw, 0.0) / (double)r;
        double Rc = 0;
        for (int j = 0; j < c; ++j) Rc += mr[(size_t)j] / (double)r;
        Rc /= c;
        q.R.wimpy = W;
        q.R.mcera = Rc;
        // round i runs at delta_i = delta / 2^(i+1); a fixed sample uses delta
        const double dd = q.rq.delta > 0 && q.rq.delta < 1 ? q.rq.delta : 0.1;
        const double di = q.rq.fixed_r > 0 ? dd : q.rq.delta / pow(2.0, (double)(q.round + 1));
        q.R.xi = bnd::xi(Rc, W, std::min(0.25, W), c, (double)r, di);
    }
    if (q.rq.fixed_r > 0) { q.phase = ReqRun::DONE; return MANTRA_OK; }
    if (r >= q.om) { q.R.flags |= MANTRA_RES_STOP_OMEGA; q.phase = ReqRun::DONE; return MANTRA_OK; }
    if (q.R.xi <= q.rq.eps) { q.R.flags |= MANTRA_RES_STOP_XI; q.phase = ReqRun::DONE; return MANTRA_OK; }
    q.prev = q.target;
    q.issued = 0;
    q.target = std::min(bnd::next(q.target), q.om);
    return MANTRA_OK;
}

int req_finish(mantra_graph *g, ReqRun &q, mantra_result *out) {
    int rc = q.rc;
    if (rc < 0 && q.err.empty()) q.err = g_err;
    if (!rc) rc = finish_outputs(g, q.rq, q.acc, q.R.samples);
    req_release(q);
    if (!rc && q.R.n_overflow > 0)
        rc = fail(MANTRA_E_OVERFLOW, "%lld sampled pairs saturated", (long long)q.R.n_overflow);
    if (rc == MANTRA_E_OVERFLOW && q.rq.node_bc)
        for (int64_t v = 0; v < g->n_total; ++v) q.rq.node_bc[v] = NAN;
    if (rc == MANTRA_E_OVERFLOW && q.edges)
        for (int64_t i = 0; i < g->m_in; ++i) q.rq.edge_bc[i] = NAN;
    q.R.latency_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - q.t_start).count();
    q.R.status = rc;
    q.R.node_bc = q.rq.node_bc;
    q.R.edge_bc = q.edges ? q.rq.edge_bc : nullptr;
    if (rc < 0 && q.rc == MANTRA_OK) q.err = g_err;
    q.rc = rc;
    if (out) *out = q.R;
    return rc;
}

// Algorithm 1 (or a fixed sample) for one request, blocking: each phase is
// one launch
static int run_request(mantra_graph *g, const mantra_request &rq, mantra_result *res) {
    ReqRun q;
    q.rq = rq;
    timing_reset(g);
    int rc = req_begin(g, q);
    while (!rc && q.phase != ReqRun::DONE) {
        LaunchSpec sp;
        const int64_t cnt = req_pending(q);
        sp.reqs.push_back(req_slice(q, cnt, 0));
        sp.npairs = cnt;
        sp.mode = sp.reqs[0].mode;
        // progressive rounds: one graph, captured for the largest round
        RoundGraph *rg = nullptr;
        if (g->graph_rounds && !g->per_pair && q.phase == ReqRun::ROUND && q.rq.fixed_r <= 0) {
            rg = &q.rg;
            if (!rg->exec) { rg->cap = q.om; rg->W = q.acc.W; rg->B = q.acc.B; rg->R = q.acc.R; rg->c = q.c; }
        }
        SweepOut o;
        rc = run_sweep(g, sp, o, rg);
        timing_add(g, o);
        q.R.gpu_ms += o.ms;
        q.reduced = o.reduced;
        if (!rc) rc = req_advance(g, q);
    }
    q.rc = rc;
    return req_finish(g, q, res);
}

// ------------------------------------------------------------------ autotuner

// Times candidate launch configurations on a calibration sample of pairs
// (their own stream, so no request's pairs are touched) and keeps the
// fastest: the number of persistent workgroups (pairs in flight) and the
// order pairs are handed out in.  The arc capacity follows the slab count
// (the rest of the pool budget).  Results never depend on the choice.
static int autotune(mantra_graph *g, mantra_opt opt, int64_t sample, uint64_t seed, mantra_launch_config *best) {
    const int saved_slabs = g->user_slabs, saved_order = g->order_mode, saved_hub = g->hub_nodes;
    const int64_t saved_cap = g->user_cap;
    g->user_slabs = 0;
    g->user_cap = 0;
    g->hub_nodes = 0;
    const int full = auto_slabs(g);
    std::vector<int> slabs;
    // a grid bounded by memory (large graphs) trades pairs in flight against
    // the shared arc chunks: 3/2 and 5/4 of it leave a quarter and three
    // eighths of the budget to the chunks (pairs that find none are re-run
    // after the launch, inside the timed call), 3/4 to 3/8 of it leave more
    const int res = resident_slabs(g);
    if (full < res) {
        slabs.push_back(std::min(res, (3 * full) / 2));
        slabs.push_back(std::min(res, (5 * full) / 4));
        for (int x : {full, (3 * full) / 4, full / 2, (3 * full) / 8}) slabs.push_back(std::max(1, x));
    } else {
        for (int x : {full, (7 * full) / 8, (3 * full) / 4, (5 * full) / 8, full / 2}) slabs.push_back(std::max(1, x));
    }
    std::sort(slabs.begin(), slabs.end(), std::greater<int>());
    slabs.erase(std::unique(slabs.begin(), slabs.end()), slabs.end());
    // Candidates are compared by the sample's time.  Where memory bounds the
    // grid (large graphs), the sample is smaller than the rounds it tunes for
    // and its time would be its longest pairs': there they are compared by
    // the grid's mean busy time instead (the persistent launch's time times
    // its busy share, plus any re-runs), the sample's time at a steady state.
    // Default sample: four pairs per workgroup of the largest candidate, two
    // where memory bounds the grid.
    const bool steady = full < res;
    if (sample <= 0) sample = std::max<int64_t>((steady ? 2 : 4) * (int64_t)slabs.front(), 256);
    mantra_request rq;
    memset(&rq, 0, sizeof rq);
    rq.opt = opt;
    rq.t0 = 0;
    rq.t1 = INT32_MAX;
    rq.seed = seed;
    double best_ms = INFINITY;
    int best_slabs = full, best_order = MANTRA_ORDER_LONGEST_FIRST, best_hub = 0;
    int rc = MANTRA_OK;
    auto time_one = [&](double *ms) {
        LaunchSpec sp;
        DevReq d = make_req(rq, STREAM_BOOT, 0, 0, sample, nullptr, 0);
        d.graph = g->G == 1 ? 0 : -1;
        d.per_graph = (sample + g->G - 1) / g->G;
        sp.reqs.push_back(d);
        sp.npairs = g->G == 1 ? sample : d.per_graph * g->G;
        SweepOut o;
        const int r = run_sweep(g, sp, o);
        *ms = steady ? o.first_ms * o.balance + (o.ms - o.first_ms) : o.ms;
        return r;
    };
    for (int order : {MANTRA_ORDER_LONGEST_FIRST, MANTRA_ORDER_DRAWN}) {
        // the order only shapes the tail of a launch, which the steady-state
        // comparison leaves out: longest first there
        if (steady && order != MANTRA_ORDER_LONGEST_FIRST) continue;
        for (int ns : slabs) {
            g->user_slabs = ns;
            g->order_mode = order;
            double ms = 0;
            if ((rc = time_one(&ms))) break;
            if (ms < best_ms) { best_ms = ms; best_slabs = ns; best_order = order; }
        }
        if (rc) break;
    }
    // hub nodes' state in LDS.  Where residency bounds the grid: 256 of
    // them at the best grid, then 256, 512 and 1,024 at the grids resident
    // with that much more LDS per workgroup (all and 7/8 of them).  Where
    // memory bounds it (few workgroups per CU, LDS to spare): 1,024, 2,048
    // and 4,096 at the best grid, or at the grid still resident with them.
    if (!rc) {
        g->order_mode = best_order;
        std::vector<std::pair<int, int>> trials;
        if (!steady) {
            trials.push_back({256, best_slabs});
            for (int K : {256, 512, 1024}) {
                g->hub_nodes = K;
                g->user_slabs = 0;
                const int rk = auto_slabs(g);
                for (int ns : {rk, (7 * rk) / 8})
                    if (ns >= 1 && (K != 256 || ns != best_slabs)) trials.push_back({K, ns});
            }
        } else {
            for (int K : {1024, 2048, 4096}) {
                g->hub_nodes = K;
                trials.push_back({K, std::min(best_slabs, resident_slabs(g))});
            }
        }
        for (const auto &tr : trials) {
            g->hub_nodes = tr.first;
            g->user_slabs = tr.second;
            double ms = 0;
            if ((rc = time_one(&ms))) break;
            if (ms < best_ms) { best_ms = ms; best_hub = tr.first; best_slabs = tr.second; }
        }
    }
    if (rc) {
        g->user_slabs = saved_slabs;
        g->user_cap = saved_cap;
        g->order_mode = saved_order;
        g->hub_nodes = saved_hub;
        return rc;
    }
    g->user_cap = 0;
    g->order_mode = best_order;
    g->hub_nodes = best_hub;
    g->user_slabs = 0;
    if (auto_slabs(g) != best_slabs) g->user_slabs = best_slabs;
    if (best) {
        best->n_slabs = best_slabs;
        best->arc_cap = own_cap(g);
        best->no_arc_chunks = g->no_chunks;
        best->arc_chunks = g->max_chunks;
        best->order = best_order;
        best->graph_rounds = g->graph_rounds;
        best->per_pair_launch = g->per_pair;
        best->hub_nodes = hub_nodes(g);
        best->wide_counts = g->wide_mode;
    }
    return MANTRA_OK;
}

}  // namespace mantra

// ------------------------------------------------------------------ C ABI

using namespace mantra;

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

void mantra_graph_destroy(mantra_graph *g) {
    if (!g) return;
    serve_stop(g);
    hipSetDevice(g->device);
    if (g->st) hipStreamSynchronize(g->st);
    g->pool.release();
    g->pool_big.release();
    g->wide.release();
    hipFree(g->dwide);
    hipFree(g->dU); hipFree(g->dV); hipFree(g->dT); hipFree(g->dout_t); hipFree(g->din_t);
    hipFree(g->dout_off); hipFree(g->din_off); hipFree(g->dseg_eoff); hipFree(g->dseg_noff); hipFree(g->dperm);
    hipFree(g->din2k); hipFree(g->dout);
    hipFree(g->dwork); hipFree(g->dstats); hipFree(g->dretry); hipFree(g->dpart); hipFree(g->dreqs);
    hipFree(g->dbucket); hipFree(g->dorder); hipFree(g->dhist); hipFree(g->dnp);
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

int mantra_set_launch(mantra_graph *g, const mantra_launch_config *cfg) {
    if (!g || !cfg) return fail(MANTRA_E_INVALID, "graph or config is NULL");
    if (cfg->n_slabs < 0 || cfg->arc_cap < 0 || cfg->arc_chunks < 0)
        return fail(MANTRA_E_INVALID, "negative launch setting");
    if (cfg->order != MANTRA_ORDER_LONGEST_FIRST && cfg->order != MANTRA_ORDER_DRAWN)
        return fail(MANTRA_E_INVALID, "unknown pair order %d", cfg->order);
    if (cfg->hub_nodes < 0 || cfg->hub_nodes > 4096) return fail(MANTRA_E_INVALID, "hub_nodes outside 0..4096");
    if (cfg->wide_counts < MANTRA_WIDE_NONE || cfg->wide_counts > MANTRA_WIDE_ALL)
        return fail(MANTRA_E_INVALID, "unknown wide_counts %d", cfg->wide_counts);
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->user_slabs != cfg->n_slabs || g->user_cap != cfg->arc_cap || g->no_chunks != (cfg->no_arc_chunks ? 1 : 0) ||
        g->max_chunks != cfg->arc_chunks)
        g->pool.release();
    g->user_slabs = cfg->n_slabs;
    g->user_cap = cfg->arc_cap;
    g->no_chunks = cfg->no_arc_chunks ? 1 : 0;
    g->max_chunks = cfg->arc_chunks;
    g->order_mode = cfg->order;
    g->graph_rounds = cfg->graph_rounds ? 1 : 0;
    g->per_pair = cfg->per_pair_launch ? 1 : 0;
    g->hub_nodes = cfg->hub_nodes;
    g->wide_mode = cfg->wide_counts;
    return MANTRA_OK;
}

int mantra_autotune(mantra_graph *g, mantra_opt opt, int64_t sample_pairs, uint64_t seed, mantra_launch_config *best) {
    if (!g) return fail(MANTRA_E_INVALID, "graph is NULL");
    if (opt < MANTRA_SH || opt > MANTRA_PFM) return fail(MANTRA_E_INVALID, "unknown optimality %d", (int)opt);
    if (sample_pairs < 0) return fail(MANTRA_E_INVALID, "negative sample size");
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->per_pair) return fail(MANTRA_E_INVALID, "the per-pair launch form has nothing to tune");
    timing_reset(g);
    return autotune(g, opt, sample_pairs, seed, best);
}

int mantra_get_launch(const mantra_graph *g, mantra_launch_config *cfg) {
    if (!g || !cfg) return fail(MANTRA_E_INVALID, "graph or config is NULL");
    cfg->n_slabs = auto_slabs(g);
    cfg->arc_cap = own_cap(g);
    cfg->no_arc_chunks = g->no_chunks;
    cfg->arc_chunks = g->max_chunks;
    cfg->order = g->order_mode;
    cfg->graph_rounds = g->graph_rounds;
    cfg->per_pair_launch = g->per_pair;
    cfg->hub_nodes = hub_nodes(g);
    cfg->wide_counts = g->wide_mode;
    return MANTRA_OK;
}

int mantra_debug_stamps(mantra_graph *g, uint32_t serial) {
    if (!g) return fail(MANTRA_E_INVALID, "graph is NULL");
    std::lock_guard<std::mutex> lk(g->mu);
    hipSetDevice(g->device);
    int rc = pool_for(g, auto_slabs(g));
    if (rc) return rc;
    std::vector<u32> h((size_t)g->pool.nslabs * 4, 0u);
    for (size_t i = 0; i < (size_t)g->pool.nslabs; ++i) h[4 * i] = serial;
    HIPCHK(hipMemcpy(g->pool.hdr, h.data(), sizeof(u32) * h.size(), hipMemcpyHostToDevice));
    g->pool.serial_hi = serial;
    if (g->wide.nslabs) {
        std::vector<u32> w((size_t)g->wide.nslabs * 4, 0u);
        for (size_t i = 0; i < (size_t)g->wide.nslabs; ++i) w[4 * i] = serial;
        HIPCHK(hipMemcpy(g->wide.hdr, w.data(), sizeof(u32) * w.size(), hipMemcpyHostToDevice));
        g->wide.serial_hi = serial;
    }
    return MANTRA_OK;
}

int mantra_last_timing(const mantra_graph *g, double *sweep_ms, int64_t *launches, int64_t *window_edges,
                       int64_t *arcs, int64_t *touched_nodes, int64_t *touched_edges, double *balance,
                       int64_t *live_batches, int64_t *skipped_batches, double *forward_share) {
    if (!g) return fail(MANTRA_E_INVALID, "graph is NULL");
    g_err.clear();
    if (sweep_ms) *sweep_ms = g->last_ms;
    if (launches) *launches = g->last_launches;
    if (window_edges) *window_edges = g->last_W;
    if (arcs) *arcs = g->last_arcs;
    if (touched_nodes) *touched_nodes = g->last_tn;
    if (touched_edges) *touched_edges = g->last_te;
    if (balance) *balance = g->last_ms > 0 ? g->last_busy_ms / g->last_ms : 1.0;
    if (live_batches) *live_batches = g->last_live;
    if (skipped_batches) *skipped_batches = g->last_dead;
    if (forward_share) {
        const double all = (double)g->last_fwd_ticks + (double)g->last_rev_ticks;
        *forward_share = all > 0 ? (double)g->last_fwd_ticks / all : 0.0;
    }
    return MANTRA_OK;
}

}  // extern "C"

// explicit pairs (s[q], z[q]) in one launch: records and optional dense f;
// mode MODE_PAIRS (f = N / sigma) or MODE_TRK (f = visits of the walk drawn
// with seed)
static int explicit_pairs(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r, const int32_t *graph,
                          const int32_t *s, const int32_t *z, uint64_t seed, int mode, mantra_pair_record *out,
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
        if (mode == MODE_RTB) {
            if (s[q] < 0 || s[q] >= ng) return fail(MANTRA_E_INVALID, "source %lld: %d not a node of graph %d",
                                                    (long long)q, s[q], gi);
            continue;
        }
        if (s[q] < 0 || s[q] >= ng || z[q] < 0 || z[q] >= ng || s[q] == z[q])
            return fail(MANTRA_E_INVALID, "pair %lld: (%d, %d) not two distinct nodes of graph %d", (long long)q,
                        s[q], z[q], gi);
    }
    if (node_f && (double)r * (double)g->n_total > 4e9) return fail(MANTRA_E_INVALID, "node_f too large");
    if (edge_f && (double)r * (double)g->m > 4e9) return fail(MANTRA_E_INVALID, "edge_f too large");
    std::lock_guard<std::mutex> lk(g->mu);
    hipSetDevice(g->device);
    timing_reset(g);
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
            zi[(size_t)q] = mode == MODE_RTB ? 0 : g->perm[(size_t)(b + z[q])] - b;
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
    rq.opt = opt; rq.t0 = t0; rq.t1 = t1; rq.seed = seed;
    if (mode == MODE_TRK) rq.flags |= MANTRA_F_TRK;
    if (mode == MODE_RTB) rq.flags |= MANTRA_F_RTB;
    norm_window(rq);
    sp.reqs.push_back(make_req(rq, STREAM_PAIR, 0, 0, r, nullptr, 0));
    sp.npairs = r;
    sp.mode = mode;
    sp.dpg = dpg; sp.dps = dps; sp.dpz = dpz; sp.drec = drec; sp.dnode_f = dnf; sp.dedge_f = def;
    SweepOut so;
    rc = run_sweep(g, sp, so);
    timing_add(g, so);
    if (!rc) {
        if (hipMemcpy(out, drec, (size_t)r * 24, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(MANTRA_E_INTERNAL, "copy records");
        if (!rc && node_f) rc = copy_out(g, node_f, dnf, g->dperm, g->n_total, g->n_total, r, 0.0);
        if (!rc && edge_f) rc = copy_out(g, edge_f, def, g->din2k, g->m_in, g->m, r, 0.0);
        if (!rc && hipStreamSynchronize(g->st) != hipSuccess) rc = fail(MANTRA_E_INTERNAL, "copy per-pair outputs");
    }
    cleanup();
    return rc;
}

extern "C" {

int mantra_count_pairs(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r,
                       const int32_t *graph, const int32_t *s, const int32_t *z, mantra_pair_record *out,
                       double *node_f, double *edge_f) {
    return explicit_pairs(g, opt, t0, t1, r, graph, s, z, 0, MODE_PAIRS, out, node_f, edge_f);
}

int mantra_sample_paths(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r, const int32_t *graph,
                        const int32_t *s, const int32_t *z, uint64_t seed, mantra_pair_record *out, double *node_f,
                        double *edge_f) {
    return explicit_pairs(g, opt, t0, t1, r, graph, s, z, seed, MODE_TRK, out, node_f, edge_f);
}

int mantra_source_dependencies(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r,
                               const int32_t *graph, const int32_t *s, mantra_pair_record *out, double *node_f,
                               double *edge_f) {
    return explicit_pairs(g, opt, t0, t1, r, graph, s, s, 0, MODE_RTB, out, node_f, edge_f);
}

int mantra_run(mantra_graph *g, const mantra_request *req, mantra_result *out) {
    if (!g || !req) return fail(MANTRA_E_INVALID, "graph or request is NULL");
    std::lock_guard<std::mutex> lk(g->mu);
    hipSetDevice(g->device);
    return run_request(g, *req, out);
}

int mantra_estimate(mantra_graph *g, mantra_opt opt, double eps, double delta, uint64_t seed,
                    mantra_result *out) {
    if (!out || !out->node_bc) return fail(MANTRA_E_INVALID, "mantra_estimate needs out->node_bc");
    mantra_request rq;
    memset(&rq, 0, sizeof rq);
    rq.opt = opt; rq.t0 = 0; rq.t1 = INT32_MAX; rq.eps = eps; rq.delta = delta; rq.seed = seed; rq.c = 25;
    rq.node_bc = out->node_bc;
    rq.edge_bc = out->edge_bc;
    if (out->edge_bc) rq.flags |= MANTRA_F_EDGE_BC;
    return mantra_run(g, &rq, out);
}

int mantra_distances(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r, uint64_t seed,
                     double tau, uint64_t *hist, int32_t hist_len, mantra_distance_result *out) {
    if (!g || !out) return fail(MANTRA_E_INVALID, "graph or result is NULL");
    if (opt < MANTRA_SH || opt > MANTRA_PFM) return fail(MANTRA_E_INVALID, "unknown optimality %d", (int)opt);
    if (g->G != 1) return fail(MANTRA_E_INVALID, "distances need a single graph");
    if (g->n_total < 2) return fail(MANTRA_E_INVALID, "distances need n >= 2");
    if (r < 1 || r > INT32_MAX) return fail(MANTRA_E_INVALID, "r = %lld outside 1..2^31-1", (long long)r);
    if (!(tau >= 0.0 && tau <= 1.0)) return fail(MANTRA_E_INVALID, "tau must be in [0, 1]");
    if (hist_len < 0 || (hist_len > 0 && !hist)) return fail(MANTRA_E_INVALID, "bad hist buffer");
    std::lock_guard<std::mutex> lk(g->mu);
    hipSetDevice(g->device);
    timing_reset(g);
    // every finite distance has its own bin: 0..kHInf-1, then the largest
    const int64_t nb = (int64_t)kHInf;
    u64 *dbuf = nullptr;
    HIPCHK(dalloc(&dbuf, (size_t)(nb + 1 + RS_N)));
    u64 *dhist = dbuf, *drs = dbuf + nb + 1;
    int rc = MANTRA_OK;
    if (hipMemsetAsync(dbuf, 0, sizeof(u64) * (size_t)(nb + 1 + RS_N), g->st) != hipSuccess)
        rc = fail(MANTRA_E_INTERNAL, "clear distance counts");
    mantra_request rq;
    memset(&rq, 0, sizeof rq);
    rq.opt = opt; rq.t0 = t0; rq.t1 = t1; rq.seed = seed;
    norm_window(rq);
    LaunchSpec sp;
    DevReq d = make_req(rq, STREAM_SRC, 0, 0, r, nullptr, 0);
    d.mode = MODE_DISTANCES;
    d.hist_len = (int32_t)nb;
    d.hist = dhist;
    d.rstat = drs;
    sp.reqs.push_back(d);
    sp.npairs = r;
    sp.mode = MODE_DISTANCES;
    SweepOut so;
    std::vector<u64> h((size_t)nb + 1);
    u64 rs[RS_N];
    if (!rc) rc = run_sweep(g, sp, so);
    if (!rc) {
        timing_add(g, so);
        if (hipMemcpy(h.data(), dhist, sizeof(u64) * (size_t)(nb + 1), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(rs, drs, sizeof rs, hipMemcpyDeviceToHost) != hipSuccess)
            rc = fail(MANTRA_E_INTERNAL, "copy distance counts");
    }
    hipFree(dbuf);
    if (rc) return rc;
    if (rs[RS_HOPS]) return fail(MANTRA_E_LIMIT, "%llu sources reached a distance above 65534",
                                 (unsigned long long)rs[RS_HOPS]);
    // Algorithm 2's closing formulas on exact integer sums of the counts
    const int32_t dlb = (int32_t)h[(size_t)nb];
    unsigned __int128 tot = 0, sh = 0, shm1 = 0;
    for (int64_t k = 1; k <= dlb; ++k) {
        tot += h[(size_t)k];
        sh += (unsigned __int128)h[(size_t)k] * (u64)k;
        shm1 += (unsigned __int128)h[(size_t)k] * (u64)(k - 1);
    }
    const double n = (double)g->n_total, rr = (double)r;
    memset(out, 0, sizeof *out);
    out->sources = r;
    out->reached_pairs = (int64_t)tot;
    out->d_lb = dlb;
    out->d_tau = -1;
    if (tot) {
        // D_tau: the first h whose share of the reachable pairs is >= tau
        unsigned __int128 cum = 0;
        for (int64_t k = 0; k <= dlb; ++k) {
            cum += h[(size_t)k];
            if ((double)cum / (double)tot >= tau) { out->d_tau = (int32_t)k; break; }
        }
        out->psi = (double)sh / (double)tot;
    }
    out->zeta = (double)tot / (rr * (n - 1.0));
    out->rho = (double)shm1 / (rr * (n - 1.0));
    out->window_edges = (int64_t)rs[RS_WINDOW];
    out->gpu_ms = so.ms;
    for (int32_t k = 0; k < hist_len; ++k) hist[k] = 0;
    for (int64_t k = 0; k <= dlb && hist_len > 0; ++k) hist[std::min<int64_t>(k, hist_len - 1)] += h[(size_t)k];
    return MANTRA_OK;
}

}  // extern "C"

// serving lives in mantra_serve.hip
