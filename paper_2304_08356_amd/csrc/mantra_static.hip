// The per-pair records of mantra_count_pairs for callers that cannot
// allocate device memory: every buffer the sweep needs beyond the graph
// (the slabs' node state and arc records, the launch counters, the pairs
// and the records) lives in one statically sized device array of this
// library, and the call makes no device allocation.
//
// The array is a file-scope __device__ variable: each GPU the library runs
// on holds its own copy from module load until the process ends.  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (the variable's name is not a device address on the host),
// fetched once per device.  Calls on one device share the array and leave
// their contents in it; the library serializes them per device, and each
// call clears (with fill kernels) everything that must start at zero.

#include "mantra_int.h"

namespace mantra {

constexpr size_t kScratchBytes = (size_t)256 << 20;  // 256 MiB per device
constexpr int kStaticMaxDevices = 64;
constexpr int kStaticMaxSlabs = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_static_mu[kStaticMaxDevices];
unsigned char *g_scratch_ptr[kStaticMaxDevices];  // device address of scratch, per device

// the device address of the current device's array (first use: looked up)
int scratch_of(int dev, unsigned char **out) {
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MANTRA_E_INTERNAL, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return MANTRA_OK;
}

// bump layout of the array, 256-byte aligned pieces
struct Carve {
    size_t used = 0;
    template <class T>
    size_t take(size_t count) {
        const size_t at = (used + 255) & ~(size_t)255;
        used = at + sizeof(T) * (count ? count : 1);
        return at;
    }
};

// the slab pieces of ns slabs for graph g, own arc room cap (offsets into the array)
struct SlabOffsets {
    size_t F, N, AG, touched, arcs, XS, hdr, BM;
};
SlabOffsets carve_slabs(Carve &c, const mantra_graph *g, size_t ns, int64_t cap) {
    SlabOffsets o;
    const size_t n = (size_t)g->nmax, gm = (size_t)g->gmax;
    o.F = c.take<u64>(ns * n * 2);
    o.N = c.take<u64>(ns * n);
    o.AG = c.take<u64>(ns * gm * 2);
    o.touched = c.take<int32_t>(ns * n);
    o.arcs = c.take<u64>(ns * (size_t)cap * 4);
    o.XS = c.take<u64>(ns * gm * 2);
    o.hdr = c.take<u32>(ns * 4);
    o.BM = c.take<unsigned char>(ns * node_bytes_per_slab(g->nmax));
    return o;
}

}  // namespace
}  // namespace mantra

using namespace mantra;

extern "C" {

int mantra_count_pairs_static(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r,
                              const int32_t *graph, const int32_t *s, const int32_t *z, mantra_pair_record *out) {
    if (!g) return fail(MANTRA_E_INVALID, "graph is NULL");
    if (r < 0 || (r > 0 && (!s || !z || !out))) return fail(MANTRA_E_INVALID, "bad pair arrays");
    if (opt < MANTRA_SH || opt > MANTRA_PFM) return fail(MANTRA_E_INVALID, "unknown optimality %d", (int)opt);
    if (r == 0) return MANTRA_OK;
    if (r > INT32_MAX) return fail(MANTRA_E_INVALID, "too many pairs");
    if (g->device < 0 || g->device >= kStaticMaxDevices) return fail(MANTRA_E_INVALID, "device %d", g->device);
    for (int64_t q = 0; q < r; ++q) {
        const int32_t gi = graph ? graph[q] : 0;
        if (gi < 0 || gi >= g->G) return fail(MANTRA_E_INVALID, "pair %lld: graph %d", (long long)q, gi);
        const int32_t ng = g->seg_noff[gi + 1] - g->seg_noff[gi];
        if (s[q] < 0 || s[q] >= ng || z[q] < 0 || z[q] >= ng || s[q] == z[q])
            return fail(MANTRA_E_INVALID, "pair %lld: (%d, %d) not two distinct nodes of graph %d", (long long)q,
                        s[q], z[q], gi);
    }
    // Layout: the request, counters and pairs, then as many slabs (up to 64)
    // as the rest holds, each with room for an arc per edge of the graph
    // (a pair never records more), so that no pair needs a re-run.
    const int64_t cap = g->m + 1;
    Carve head;
    const size_t o_req = head.take<DevReq>(1);
    const size_t o_work = head.take<u32>(1);
    const size_t o_retry = head.take<int32_t>(1 + (size_t)r);
    const size_t o_stats = head.take<u64>(kStats);
    const size_t o_ps = head.take<int32_t>((size_t)r);
    const size_t o_pz = head.take<int32_t>((size_t)r);
    const size_t o_pg = head.take<int32_t>((size_t)r);
    const size_t o_rec = head.take<mantra_pair_record>((size_t)r);
    Carve one = head;
    carve_slabs(one, g, 1, cap);
    if (one.used > kScratchBytes)
        return fail(MANTRA_E_TOO_LARGE, "%lld pairs and one slab of this graph need %zu bytes, the static array holds %zu",
                    (long long)r, one.used, kScratchBytes);
    size_t ns = 1;
    while (ns < (size_t)kStaticMaxSlabs && ns < (size_t)r) {
        Carve t = head;
        carve_slabs(t, g, ns + 1, cap);
        if (t.used > kScratchBytes) break;
        ++ns;
    }
    Carve body = head;
    const SlabOffsets so = carve_slabs(body, g, ns, cap);

    std::lock_guard<std::mutex> lk(g->mu);
    std::lock_guard<std::mutex> sk(g_static_mu[g->device]);
    hipSetDevice(g->device);
    unsigned char *base = nullptr;
    int rc = scratch_of(g->device, &base);
    if (rc) return rc;
    timing_reset(g);
    // inputs: pairs in internal node ids
    {
        std::vector<int32_t> si((size_t)r), zi((size_t)r), gi((size_t)r);
        for (int64_t q = 0; q < r; ++q) {
            const int32_t gq = graph ? graph[q] : 0;
            const int32_t b = g->seg_noff[gq];
            si[(size_t)q] = g->perm[(size_t)(b + s[q])] - b;
            zi[(size_t)q] = g->perm[(size_t)(b + z[q])] - b;
            gi[(size_t)q] = gq;
        }
        HIPCHK(hipMemcpyAsync(base + o_ps, si.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice, g->st));
        HIPCHK(hipMemcpyAsync(base + o_pz, zi.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice, g->st));
        HIPCHK(hipMemcpyAsync(base + o_pg, gi.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice, g->st));
        DevReq d;
        memset(&d, 0, sizeof d);
        d.opt = opt;
        d.t0 = t0;
        d.t1 = t1;
        if (d.t1 < d.t0) { d.t0 = 0; d.t1 = INT32_MAX; }
        d.stream = STREAM_PAIR;
        d.count = r;
        d.per_graph = r;
        d.mode = MODE_PAIRS;
        HIPCHK(hipMemcpyAsync(base + o_req, &d, sizeof d, hipMemcpyHostToDevice, g->st));
        // the copies read host memory that lives until the synchronisation
        HIPCHK(hipStreamSynchronize(g->st));
    }
    // what must start at zero (the previous call's contents are still there):
    // pair tags and counts, N, slab serials, counters
    const size_t n = (size_t)g->nmax;
    HIPCHK(mantra_launch_fill(reinterpret_cast<u64 *>(base + so.F), 0ull, (int64_t)(ns * n * 2), g->st));
    HIPCHK(mantra_launch_fill(reinterpret_cast<u64 *>(base + so.N), 0ull, (int64_t)(ns * n), g->st));
    HIPCHK(mantra_launch_fill(reinterpret_cast<u64 *>(base + so.hdr), 0ull, (int64_t)(ns * 2), g->st));
    HIPCHK(mantra_launch_clear(reinterpret_cast<u32 *>(base + o_work), reinterpret_cast<u32 *>(base + o_retry),
                               nullptr, reinterpret_cast<u64 *>(base + o_stats), g->st));
    LaunchArgs a;
    memset(&a, 0, sizeof a);
    a.g = g->dev();
    a.sl.F = reinterpret_cast<u64 *>(base + so.F);
    a.sl.N = reinterpret_cast<u64 *>(base + so.N);
    a.sl.AG = reinterpret_cast<u64 *>(base + so.AG);
    a.sl.touched = reinterpret_cast<int32_t *>(base + so.touched);
    a.sl.arcs = reinterpret_cast<u64 *>(base + so.arcs);
    a.sl.XS = reinterpret_cast<u64 *>(base + so.XS);
    a.sl.hdr = reinterpret_cast<u32 *>(base + so.hdr);
    a.sl.BM = node_bytes_per_slab(g->nmax) ? base + so.BM : nullptr;
    a.sl.T = nullptr;
    a.sl.xarcs = nullptr;
    a.sl.xfree = nullptr;
    a.sl.xtab = nullptr;
    a.sl.xwords = 0;
    a.sl.xmax = 0;
    a.sl.nmax = g->nmax;
    a.sl.cap = cap;
    a.sl.gmax = g->gmax;
    a.reqs = reinterpret_cast<const DevReq *>(base + o_req);
    a.nreq = 1;
    a.lds_bitmap = lds_bitmap_ok(g->nmax);
    a.hub_nodes = 0;
    a.npairs = r;
    a.npairs_dev = nullptr;
    a.qbase = 0;
    a.pg = graph ? reinterpret_cast<const int32_t *>(base + o_pg) : nullptr;
    a.ps = reinterpret_cast<const int32_t *>(base + o_ps);
    a.pz = reinterpret_cast<const int32_t *>(base + o_pz);
    a.pq = nullptr;
    a.rec = base + o_rec;
    a.node_f = nullptr;
    a.edge_f = nullptr;
    a.work = reinterpret_cast<u32 *>(base + o_work);
    a.stats = reinterpret_cast<u64 *>(base + o_stats);
    a.retry = reinterpret_cast<int32_t *>(base + o_retry);
    a.wide = nullptr;  // saturated pairs are reported (MANTRA_REC_OVERFLOW)
    a.wide_fm = 0;
    size_t lb = mantra_tab_lds_bytes();
    if (a.lds_bitmap) lb += ((size_t)((g->nmax + 31) / 32) * 4 + 7) & ~(size_t)7;
    HIPCHK(hipEventRecord(g->ev0, g->st));
    HIPCHK(mantra_launch_sweep(&a, (int)ns, lb, g->st));
    HIPCHK(hipEventRecord(g->ev1, g->st));
    HIPCHK(hipMemcpyAsync(out, base + o_rec, sizeof(mantra_pair_record) * r, hipMemcpyDeviceToHost, g->st));
    u64 st[kStats];
    HIPCHK(hipMemcpyAsync(st, base + o_stats, sizeof st, hipMemcpyDeviceToHost, g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
    SweepOut o;
    memcpy(o.st, st, sizeof st);
    o.ms = ms;
    o.first_ms = ms;
    o.launches = 1;
    const u64 span = st[10] - ~st[11];
    o.balance = span ? (double)st[9] / ((double)ns * (double)span) : 1.0;
    timing_add(g, o);
    if (st[5]) return fail(MANTRA_E_INTERNAL, "%llu pairs outgrew an arc buffer of every edge", (unsigned long long)st[5]);
    if (st[6]) return fail(MANTRA_E_INTERNAL, "%llu pairs failed flow conservation", (unsigned long long)st[6]);
    return MANTRA_OK;
}

}  // extern "C"
