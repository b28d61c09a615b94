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

struct FwdLds {               // forward tables (per batch)
    u64 fw_key[kFwN];         // stamp<<32 | node
    u32 fw_run[kFwN];         // run slot holding the node's committed state
    u32 rt_d[kC];             // per run: min hop candidate
    u32 rt_nh[kC];            // per run: committed h
    u32 rt_ok[kC];            // per run: committed (useful)
    u64 rt_c[kC];             // per run: count sum
    u64 rt_nS[kC];            // per run: committed S
};
struct RevLds {               // reverse table (per batch): tail state by node
    u64 tb_key[kFwN];
    u64 tb_acc[kFwN];
    u32 tb_lvl[kFwN];         // bit 31: valid
};
union TabLds { FwdLds f; RevLds r; };

__device__ __forceinline__ u32 hslot(u32 node) { return (node * 2654435761u) >> (32 - 9); }
static_assert(kFwN == 512, "hslot assumes 512 slots");

// lookup node in a stamped open-addressing table; -1 if absent
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
        u64 old = atomicCAS((unsigned long long *)&keys[sl], (unsigned long long)k,
                            (unsigned long long)want);
        if (old == k) { *fresh = 1; return (int)sl; }
        // someone claimed it: re-examine the same slot
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
    u32 tag;
    bool level;            // sh / sfm: hop levels matter
};

struct Slab {
    u64 *F, *R, *N, *AG, *arcs, *XS;
    u32 *AGF, *hdr;
    int32_t *touched;
};

struct FwdOut {
    bool reached;
    u32 zh;
    u64 zS;
    int32_t t_arr;
    int64_t arcs;
    int64_t swept;
    u32 flags;
};

__device__ __forceinline__ bool bm_test(const u32 *bm, int32_t v) { return (bm[v >> 5] >> (v & 31)) & 1u; }

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

// ------------------------------------------------------------ forward: big tick
// A tick with more edges than one batch: aggregation by head through the
// slab's global per-node scratch (AG), four passes, commits after all reads.

__device__ void fwd_big_tick(const LaunchArgs &a, const Pair &P, const Slab &S, u32 *bm,
                             int64_t g0, int64_t g1, int32_t t, u32 &agstamp, FwdOut &o,
                             u32 &zh, u64 &zS, bool &zhit) {
    const int l = lane_id();
    const int32_t *U = a.g.U, *V = a.g.V;
    agstamp += 1;
    const u64 hi_key = (u64)(~agstamp) << 32;
    // pass A: tails, candidate minima, zero the sums
    for (int64_t sb = g0; sb < g1; sb += kWave) {
        int64_t idx = sb + l;
        bool act = idx < g1;
        int32_t u = act ? U[idx] : 0, v = act ? V[idx] : 0;
        bool rt = false;
        u32 hu = 0;
        u64 Su = 0;
        if (act) {
            bool maybe = a.lds_bitmap ? bm_test(bm, u) : true;
            if (maybe) {
                u64 th = S.F[2 * (int64_t)u], sv = S.F[2 * (int64_t)u + 1];
                if ((u32)th == P.tag) { rt = true; hu = (u32)(th >> 32) & 0xFFFFu; Su = sv; }
            }
        }
        bool hl = false;
        if (act) {
            S.XS[2 * (idx - g0)] = rt ? ((u64)hu | (1ull << 32)) : 0ull;
            S.XS[2 * (idx - g0) + 1] = Su;
            bool rs = (idx == g0) || V[idx - 1] != v;
            if (rs) S.AG[2 * (int64_t)v + 1] = 0ull;
            if (rt) {
                if (hu + 1 >= kHInf) hl = true;
                else atomicMin((unsigned long long *)&S.AG[2 * (int64_t)v], (unsigned long long)(hi_key | (hu + 1)));
            }
        }
        if (ballot(hl)) o.flags |= REC_HOPS_LIMIT;
    }
    __syncthreads();
    // pass B: sums over the tight tails
    for (int64_t sb = g0; sb < g1; sb += kWave) {
        int64_t idx = sb + l;
        if (idx >= g1) continue;
        u64 x0 = S.XS[2 * (idx - g0)];
        if (!(x0 >> 32)) continue;
        u32 hu = (u32)x0;
        u64 Su = S.XS[2 * (idx - g0) + 1];
        int32_t v = V[idx];
        u64 key = ld_agent(&S.AG[2 * (int64_t)v]);
        u32 d = (u32)key;
        bool tight = P.level ? (hu + 1 == d) : true;
        if (tight) glb_sat_add(&S.AG[2 * (int64_t)v + 1], Su);
    }
    __syncthreads();
    // pass C: one commit per head run
    u32 zh_new = zh;
    u64 zS_new = zS;
    bool zany = false;
    for (int64_t sb = g0; sb < g1; sb += kWave) {
        int64_t idx = sb + l;
        bool act = idx < g1;
        int32_t v = act ? V[idx] : 0;
        bool rs = act && ((idx == g0) || V[idx - 1] != v);
        bool zl = false;
        u32 nh = 0;
        u64 nS = 0;
        if (rs) {
            u64 key = ld_agent(&S.AG[2 * (int64_t)v]);
            u32 ok = 0;
            if ((key & 0xFFFFFFFF00000000ull) == hi_key) {
                u32 d = (u32)key;
                u64 c = ld_agent(&S.AG[2 * (int64_t)v + 1]);
                bool rv = false;
                u32 hv = 0;
                u64 Sv = 0;
                bool maybe = a.lds_bitmap ? bm_test(bm, v) : true;
                if (maybe) {
                    u64 th = S.F[2 * (int64_t)v], sv = S.F[2 * (int64_t)v + 1];
                    if ((u32)th == P.tag) { rv = true; hv = (u32)(th >> 32) & 0xFFFFu; Sv = sv; }
                }
                if (head_commit(P.opt, rv, hv, Sv, d, c, v, P.z, zh, &nh, &nS)) {
                    ok = agstamp;
                    S.F[2 * (int64_t)v] = (u64)P.tag | ((u64)nh << 32);
                    S.F[2 * (int64_t)v + 1] = nS;
                    if (a.lds_bitmap) atomicOr(&bm[v >> 5], 1u << (v & 31));
                    zl = (v == P.z);
                }
            }
            S.AGF[v] = ok;
        }
        u64 zm = ballot(zl);
        if (zm) {
            int zlane = __ffsll((long long)zm) - 1;
            zh_new = (u32)rl32((int)nh, zlane);
            zS_new = rl64(nS, zlane);
            zany = true;
        }
    }
    if (zany) {
        if (P.opt == OPT_SH) { if (zh_new < zh) o.t_arr = t; }
        else o.t_arr = t;
        zh = zh_new;
        zS = zS_new;
        zhit = true;
    }
    __syncthreads();
    // pass D: arcs
    for (int64_t sb = g0; sb < g1; sb += kWave) {
        int64_t idx = sb + l;
        bool rec = false;
        u64 w0 = 0, w1 = 0;
        if (idx < g1) {
            u64 x0 = S.XS[2 * (idx - g0)];
            if (x0 >> 32) {
                int32_t v = V[idx];
                if (S.AGF[v] == agstamp) {
                    u32 hu = (u32)x0;
                    u32 d = (u32)ld_agent(&S.AG[2 * (int64_t)v]);
                    if (!P.level || hu + 1 == d) {
                        rec = true;
                        w0 = (u64)(u32)idx | ((u64)hu << 32) | ((u64)d << 48);
                        w1 = S.XS[2 * (idx - g0) + 1];
                    }
                }
            }
        }
        u64 m = ballot(rec);
        if (m) {
            int64_t pos = o.arcs + mbcnt(m);
            if (rec && pos < a.sl.cap) { S.arcs[2 * pos] = w0; S.arcs[2 * pos + 1] = w1; }
            o.arcs += __popcll(m);
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------ forward sweep

__device__ void forward(const LaunchArgs &a, const Pair &P, const Slab &S, u32 *bm, FwdLds &L,
                        u32 &fstamp, u32 &agstamp, FwdOut &o) {  // fstamp: shared table stamp
    const int l = lane_id();
    const int32_t *U = a.g.U, *V = a.g.V, *T = a.g.T;
    const int opt = P.opt;
    u32 zh = kHInf;
    u64 zS = 0;
    bool zhit = false;
    bool done = false;
    int64_t b0 = P.lo;
    o.arcs = 0;
    o.flags = 0;
    o.t_arr = -1;
    while (b0 < P.hi && !done) {
        const int64_t avail = P.hi - b0;
        const int nb = avail < kC ? (int)avail : kC;
        int32_t tt[kE];
#pragma unroll
        for (int j = 0; j < kE; ++j) {
            int off = j * kWave + l;
            tt[j] = off < nb ? T[b0 + off] : INT32_MAX;
        }
        int nbat = nb;
        if (nb == kC && b0 + kC < P.hi) {
            int32_t tnext = T[b0 + kC];
            int32_t tlast = rl32(tt[kE - 1], kWave - 1);
            if (tnext == tlast) {
                int first = -1;
#pragma unroll
                for (int j = 0; j < kE; ++j) {
                    u64 m = ballot(tt[j] == tlast);
                    if (first < 0 && m) first = j * kWave + (__ffsll((long long)m) - 1);
                }
                if (first == 0) {
                    // one tick longer than a batch
                    int64_t g1 = P.hi;
                    for (int64_t i = b0 + kC; i < P.hi; i += kWave) {
                        int64_t idx = i + l;
                        u64 m = ballot(idx < P.hi && T[idx] != tlast);
                        if (m) { g1 = i + (__ffsll((long long)m) - 1); break; }
                    }
                    fwd_big_tick(a, P, S, bm, b0, g1, tlast, agstamp, o, zh, zS, zhit);
                    o.swept = g1 - P.lo;
                    b0 = g1;
                    if (o.flags & (REC_HOPS_LIMIT)) return;
                    if (o.arcs > a.sl.cap) { o.flags |= REC_ARCS_LIMIT; return; }
                    if (zhit && opt != OPT_SH) done = true;
                    continue;
                }
                nbat = first;
            }
        }
        // ---- load the batch, boundaries, runs
        int32_t uu[kE], vv[kE];
        bool in[kE], gst[kE], rst[kE];
        u64 gm[kE], rm[kE];
#pragma unroll
        for (int j = 0; j < kE; ++j) {
            int off = j * kWave + l;
            in[j] = off < nbat;
            uu[j] = in[j] ? U[b0 + off] : 0;
            vv[j] = in[j] ? V[b0 + off] : -1;
        }
#pragma unroll
        for (int j = 0; j < kE; ++j) {
            int32_t tp = __shfl_up(tt[j], 1);
            int32_t vp = __shfl_up(vv[j], 1);
            if (l == 0) {
                tp = j > 0 ? rl32(tt[j - 1], kWave - 1) : INT32_MIN;
                vp = j > 0 ? rl32(vv[j - 1], kWave - 1) : -2;
            }
            gst[j] = in[j] && (tt[j] != tp);
            rst[j] = in[j] && (gst[j] || vv[j] != vp);
            gm[j] = ballot(gst[j]);
            rm[j] = ballot(rst[j]);
        }
        int roff[kE];
        {
            int last = 0;
#pragma unroll
            for (int j = 0; j < kE; ++j) {
                u64 low = (l == kWave - 1) ? kUMax : ((2ull << l) - 1ull);
                u64 mm = rm[j] & low;
                roff[j] = mm ? (j * kWave + 63 - __clzll((long long)mm)) : last;
                if (rm[j]) last = j * kWave + 63 - __clzll((long long)rm[j]);
            }
        }
        // ---- gathers: tails (reached at batch start) and run heads
        bool rt[kE], hvr[kE];
        u32 hu[kE], hv0[kE];
        u64 su[kE], sv0[kE];
#pragma unroll
        for (int j = 0; j < kE; ++j) {
            rt[j] = false; hu[j] = 0; su[j] = 0;
            hvr[j] = false; hv0[j] = kHInf; sv0[j] = 0;
            if (in[j] && (a.lds_bitmap ? bm_test(bm, uu[j]) : true)) {
                u64 th = S.F[2 * (int64_t)uu[j]], sv = S.F[2 * (int64_t)uu[j] + 1];
                if ((u32)th == P.tag) { rt[j] = true; hu[j] = (u32)(th >> 32) & 0xFFFFu; su[j] = sv; }
            }
            if (rst[j] && (a.lds_bitmap ? bm_test(bm, vv[j]) : true)) {
                u64 th = S.F[2 * (int64_t)vv[j]], sv = S.F[2 * (int64_t)vv[j] + 1];
                if ((u32)th == P.tag) { hvr[j] = true; hv0[j] = (u32)(th >> 32) & 0xFFFFu; sv0[j] = sv; }
            }
            if (rst[j]) {
                int off = j * kWave + l;
                L.rt_d[off] = kHInf;
                L.rt_c[off] = 0;
                L.rt_ok[off] = 0;
            }
        }
        fstamp += 1;
        bool fw_used = false;
        __syncthreads();
        // ---- ticks of the batch in time order
        int gs = 0;
        while (gs < nbat && !done) {
            // next tick start after gs
            int ge = nbat;
            {
                int pos = gs + 1;
                for (int j = pos >> 6; j < kE; ++j) {
                    u64 m = (j == 0) ? gm[0] : (j == 1 ? gm[1] : (j == 2 ? gm[2] : gm[3]));
                    int b = (j == (pos >> 6)) ? (pos & 63) : 0;
                    m = (b >= 64) ? 0 : (m & (kUMax << b));
                    if (m) { ge = j * kWave + (__ffsll((long long)m) - 1); break; }
                }
                if (ge > nbat) ge = nbat;
            }
            const int jlo = gs >> 6, jhi = (ge - 1) >> 6;
            const int32_t t = rl32(jlo == 0 ? tt[0] : (jlo == 1 ? tt[1] : (jlo == 2 ? tt[2] : tt[3])), gs & 63);
            // step 1: forwarded tail state, candidate minima
#pragma unroll
            for (int j = 0; j < kE; ++j) {
                if (j < jlo || j > jhi) continue;
                int off = j * kWave + l;
                bool act = off >= gs && off < ge;
                if (act && fw_used) {
                    int sl = tab_find(L.fw_key, fstamp, (u32)uu[j]);
                    if (sl >= 0) {
                        u32 r = L.fw_run[sl];
                        rt[j] = true; hu[j] = L.rt_nh[r]; su[j] = L.rt_nS[r];
                    }
                }
                bool hl = act && rt[j] && hu[j] + 1 >= kHInf;
                if (act && rt[j] && !hl) atomicMin(&L.rt_d[roff[j]], hu[j] + 1);
                if (ballot(hl)) o.flags |= REC_HOPS_LIMIT;
            }
            __syncthreads();
            // step 2: count sums
#pragma unroll
            for (int j = 0; j < kE; ++j) {
                if (j < jlo || j > jhi) continue;
                int off = j * kWave + l;
                bool act = off >= gs && off < ge;
                if (act && rt[j]) {
                    bool tight = P.level ? (hu[j] + 1 == L.rt_d[roff[j]]) : true;
                    if (tight) lds_sat_add(&L.rt_c[roff[j]], su[j]);
                }
            }
            __syncthreads();
            // step 3: run heads decide and commit
            bool zl_any = false;
            u32 zh_new = zh;
            u64 zS_new = zS;
            bool any_commit = false;
#pragma unroll
            for (int j = 0; j < kE; ++j) {
                if (j < jlo || j > jhi) continue;
                int off = j * kWave + l;
                bool act = off >= gs && off < ge;
                bool lead = act && rst[j] && L.rt_d[off] != kHInf;
                bool zl = false;
                u32 nh = 0;
                u64 nS = 0;
                bool ok = false;
                if (lead) {
                    int32_t v = vv[j];
                    bool rv = hvr[j];
                    u32 hv = hv0[j];
                    u64 Sv = sv0[j];
                    if (fw_used) {
                        int sl = tab_find(L.fw_key, fstamp, (u32)v);
                        if (sl >= 0) { u32 r = L.fw_run[sl]; rv = true; hv = L.rt_nh[r]; Sv = L.rt_nS[r]; }
                    }
                    ok = head_commit(opt, rv, hv, Sv, L.rt_d[off], L.rt_c[off], v, P.z, zh, &nh, &nS);
                    if (ok) {
                        S.F[2 * (int64_t)v] = (u64)P.tag | ((u64)nh << 32);
                        S.F[2 * (int64_t)v + 1] = nS;
                        if (a.lds_bitmap) atomicOr(&bm[v >> 5], 1u << (v & 31));
                        int fresh;
                        int sl = tab_insert(L.fw_key, fstamp, (u32)v, &fresh);
                        if (sl >= 0) L.fw_run[sl] = (u32)off;
                        L.rt_nh[off] = nh;
                        L.rt_nS[off] = nS;
                        L.rt_ok[off] = 1;
                        zl = (v == P.z);
                    }
                }
                if (ballot(ok)) any_commit = true;
                u64 zm = ballot(zl);
                if (zm) {
                    int zlane = __ffsll((long long)zm) - 1;
                    zh_new = (u32)rl32((int)nh, zlane);
                    zS_new = rl64(nS, zlane);
                    zl_any = true;
                }
            }
            if (zl_any) {
                if (opt == OPT_SH) { if (zh_new < zh) o.t_arr = t; }
                else o.t_arr = t;
                zh = zh_new;
                zS = zS_new;
                zhit = true;
            }
            if (any_commit) fw_used = true;
            __syncthreads();
            // step 4: arcs of this tick
#pragma unroll
            for (int j = 0; j < kE; ++j) {
                if (j < jlo || j > jhi) continue;
                int off = j * kWave + l;
                bool act = off >= gs && off < ge;
                bool rec = false;
                u64 w0 = 0;
                if (act && rt[j] && L.rt_ok[roff[j]]) {
                    u32 d = L.rt_d[roff[j]];
                    if (!P.level || hu[j] + 1 == d) {
                        rec = true;
                        w0 = (u64)(u32)(b0 + off) | ((u64)hu[j] << 32) | ((u64)d << 48);
                    }
                }
                u64 m = ballot(rec);
                if (m) {
                    int64_t pos = o.arcs + mbcnt(m);
                    if (rec && pos < a.sl.cap) { S.arcs[2 * pos] = w0; S.arcs[2 * pos + 1] = su[j]; }
                    o.arcs += __popcll(m);
                }
            }
            o.swept = (b0 + ge) - P.lo;
            if (o.flags & REC_HOPS_LIMIT) return;
            if (o.arcs > a.sl.cap) { o.flags |= REC_ARCS_LIMIT; return; }
            if (zhit && opt != OPT_SH) done = true;
            gs = ge;
        }
        __syncthreads();
        b0 += nbat;
    }
    o.reached = zh != kHInf;
    o.zh = zh;
    o.zS = zS;
}

// ------------------------------------------------------------ reverse sweep

struct RevCtx {
    u64 sigma;
    u32 dsh;
    int64_t touched_n;
    bool ovf;
};

__device__ __forceinline__ void rev_contrib(const LaunchArgs &a, const Pair &P, const Slab &S,
                                            RevCtx &X, bool act, u64 B, u64 tc, int32_t v, u32 k) {
    // N(arc) = tail count * B(head); N(v) += N(arc); f(e) = N(arc) / sigma
    bool first = false, wrap = false;
    if (act && B) {
        u64 na = tc * B;
        if (v != P.s && v != P.z) {
            u64 old = atomicAdd((unsigned long long *)&S.N[v], (unsigned long long)na);
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
    u64 m = ballot(first);
    if (m) {
        int64_t pos = X.touched_n + mbcnt(m);
        if (first) S.touched[pos] = v;
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

__device__ void rev_big_tick(const LaunchArgs &a, const Pair &P, const Slab &S, RevCtx &X,
                             int64_t a0, int64_t a1) {
    const int l = lane_id();
    // pass A: heads read state older than this tick
    for (int64_t sb = a0; sb < a1; sb += kWave) {
        int64_t i = sb + l;
        bool act = i < a1;
        u64 w0 = act ? S.arcs[2 * i] : 0, tc = act ? S.arcs[2 * i + 1] : 0;
        u32 k = (u32)w0, hl = (u32)(w0 >> 48);
        int32_t v = act ? a.g.V[k] : 0;
        u64 B = 0;
        if (act) {
            bool valid = false;
            u32 lvl = 0;
            u64 acc = 0;
            if (v != P.z) {
                u64 th = ld_agent(&S.R[2 * (int64_t)v]);
                if ((u32)th == P.tag) { valid = true; lvl = (u32)(th >> 32) & 0xFFFFu; acc = ld_agent(&S.R[2 * (int64_t)v + 1]); }
            }
            B = head_B(P, X, v, hl, valid, lvl, acc);
            S.XS[i - a0] = B;
        }
        rev_contrib(a, P, S, X, act, B, tc, v, k);
    }
    __syncthreads();
    // pass R: reset stale tail entries
    for (int64_t sb = a0; sb < a1; sb += kWave) {
        int64_t i = sb + l;
        if (i >= a1) continue;
        u64 B = S.XS[i - a0];
        if (!B) continue;
        u64 w0 = S.arcs[2 * i];
        u32 k = (u32)w0, tl = (u32)(w0 >> 32) & 0xFFFFu;
        int32_t u = a.g.U[k];
        u32 want = P.level ? tl : 0u;
        u64 th = ld_agent(&S.R[2 * (int64_t)u]);
        if ((u32)th != P.tag || ((u32)(th >> 32) & 0xFFFFu) != want) {
            S.R[2 * (int64_t)u] = (u64)P.tag | ((u64)want << 32);
            S.R[2 * (int64_t)u + 1] = 0;
        }
    }
    __syncthreads();
    // pass C: add
    for (int64_t sb = a0; sb < a1; sb += kWave) {
        int64_t i = sb + l;
        if (i >= a1) continue;
        u64 B = S.XS[i - a0];
        if (!B) continue;
        int32_t u = a.g.U[(u32)S.arcs[2 * i]];
        atomicAdd((unsigned long long *)&S.R[2 * (int64_t)u + 1], (unsigned long long)B);
    }
    __syncthreads();
}

__device__ void reverse(const LaunchArgs &a, const Pair &P, const Slab &S, RevLds &L, u32 &rstamp,
                        int64_t narcs, RevCtx &X) {
    const int l = lane_id();
    const int32_t *U = a.g.U, *V = a.g.V, *T = a.g.T;
    int64_t ac = narcs;
    while (ac > 0) {
        int nb = ac < kC ? (int)ac : kC;
        int64_t blo = ac - nb;
        u64 w0[kE], tc[kE];
        int32_t uu[kE], vv[kE], tt[kE];
        bool in[kE];
#pragma unroll
        for (int j = 0; j < kE; ++j) {
            int off = j * kWave + l;
            in[j] = off < nb;
            w0[j] = in[j] ? S.arcs[2 * (blo + off)] : 0;
            tc[j] = in[j] ? S.arcs[2 * (blo + off) + 1] : 0;
            u32 k = (u32)w0[j];
            uu[j] = in[j] ? U[k] : 0;
            vv[j] = in[j] ? V[k] : 0;
            tt[j] = in[j] ? T[k] : INT32_MIN;
        }
        // cut at a tick boundary at the low end
        int cut = 0;
        if (blo > 0) {
            int32_t t_first = rl32(tt[0], 0);
            int32_t t_before = T[(u32)S.arcs[2 * (blo - 1)]];
            if (t_before == t_first) {
                // first offset whose time differs from t_first
                int firstdiff = -1;
#pragma unroll
                for (int j = 0; j < kE; ++j) {
                    u64 m = ballot(in[j] && tt[j] != t_first);
                    if (firstdiff < 0 && m) firstdiff = j * kWave + (__ffsll((long long)m) - 1);
                }
                if (firstdiff < 0) {
                    // the whole batch is one tick that continues below: big tick
                    int64_t a0 = 0;
                    for (int64_t i = blo - kWave; ; i -= kWave) {
                        int64_t idx = i + l;
                        bool ok = idx >= 0 && idx < blo;
                        bool diff = ok && T[(u32)S.arcs[2 * idx]] != t_first;
                        u64 m = ballot(diff);
                        if (m) { a0 = i + (63 - __clzll((long long)m)) + 1; break; }
                        if (i <= 0) { a0 = 0; break; }
                    }
                    rev_big_tick(a, P, S, X, a0, ac);
                    ac = a0;
                    continue;
                }
                cut = firstdiff;
            }
        }
        // active: offsets [cut, nb)
#pragma unroll
        for (int j = 0; j < kE; ++j) {
            int off = j * kWave + l;
            in[j] = in[j] && off >= cut;
        }
        // tick starts (ascending offsets) within [cut, nb)
        u64 gm[kE];
#pragma unroll
        for (int j = 0; j < kE; ++j) {
            int32_t tp = __shfl_up(tt[j], 1);
            int off = j * kWave + l;
            if (l == 0) tp = j > 0 ? rl32(tt[j - 1], kWave - 1) : INT32_MIN;
            gm[j] = ballot(in[j] && (off == cut || tt[j] != tp));
        }
        // pre-gather head and tail reverse state
        bool hval[kE], tval[kE];
        u32 hlvl[kE], tlvl[kE];
        u64 hacc[kE], tacc[kE];
#pragma unroll
        for (int j = 0; j < kE; ++j) {
            hval[j] = false; hlvl[j] = 0; hacc[j] = 0;
            tval[j] = false; tlvl[j] = 0; tacc[j] = 0;
            if (in[j] && vv[j] != P.z) {
                u64 th = ld_agent(&S.R[2 * (int64_t)vv[j]]);
                if ((u32)th == P.tag) { hval[j] = true; hlvl[j] = (u32)(th >> 32) & 0xFFFFu; hacc[j] = ld_agent(&S.R[2 * (int64_t)vv[j] + 1]); }
            }
            if (in[j]) {
                u64 th = ld_agent(&S.R[2 * (int64_t)uu[j]]);
                if ((u32)th == P.tag) { tval[j] = true; tlvl[j] = (u32)(th >> 32) & 0xFFFFu; tacc[j] = ld_agent(&S.R[2 * (int64_t)uu[j] + 1]); }
            }
        }
        rstamp += 1;
        bool used = false;
        __syncthreads();
        // ticks in descending time: walk tick starts from the top
        int ge = nb;
        while (ge > cut) {
            // start of the tick that ends at ge: highest tick start < ge
            int gs = cut;
            {
                int pos = ge - 1;
                for (int j = pos >> 6; j >= 0; --j) {
                    u64 m = (j == 0) ? gm[0] : (j == 1 ? gm[1] : (j == 2 ? gm[2] : gm[3]));
                    int b = (j == (pos >> 6)) ? (pos & 63) : 63;
                    m &= (b == 63) ? kUMax : ((2ull << b) - 1ull);
                    if (m) { gs = j * kWave + 63 - __clzll((long long)m); break; }
                }
            }
            const int jlo = gs >> 6, jhi = (ge - 1) >> 6;
            u64 Bv[kE];
            // step A: heads
#pragma unroll
            for (int j = 0; j < kE; ++j) {
                Bv[j] = 0;
                if (j < jlo || j > jhi) continue;
                int off = j * kWave + l;
                bool act = off >= gs && off < ge;
                if (act) {
                    bool valid = hval[j];
                    u32 lvl = hlvl[j];
                    u64 acc = hacc[j];
                    if (used && vv[j] != P.z) {
                        int sl = tab_find(L.tb_key, rstamp, (u32)vv[j]);
                        if (sl >= 0) { u32 x = L.tb_lvl[sl]; valid = (x >> 31) != 0; lvl = x & 0xFFFFu; acc = L.tb_acc[sl]; }
                    }
                    Bv[j] = head_B(P, X, vv[j], (u32)(w0[j] >> 48), valid, lvl, acc);
                }
                rev_contrib(a, P, S, X, act, Bv[j], tc[j], vv[j], (u32)w0[j]);
            }
            // step T1: tail entries
            bool anyB = false;
            int tsl[kE];
#pragma unroll
            for (int j = 0; j < kE; ++j) {
                tsl[j] = -1;
                if (j < jlo || j > jhi) continue;
                if (Bv[j]) {
                    int fresh;
                    tsl[j] = tab_insert(L.tb_key, rstamp, (u32)uu[j], &fresh);
                    if (fresh) {
                        L.tb_lvl[tsl[j]] = tval[j] ? ((tlvl[j] & 0xFFFFu) | 0x80000000u) : 0u;
                        L.tb_acc[tsl[j]] = tval[j] ? tacc[j] : 0ull;
                    }
                }
                if (ballot(Bv[j] != 0)) anyB = true;
            }
            if (anyB) {
                used = true;
                __syncthreads();
                // step T2: level resets (identical writes for one node)
#pragma unroll
                for (int j = 0; j < kE; ++j) {
                    if (tsl[j] < 0) continue;
                    u32 want = P.level ? ((u32)(w0[j] >> 32) & 0xFFFFu) : 0u;
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
                }
                __syncthreads();
            }
            ge = gs;
        }
        // write back the tail table
        if (used) {
            for (int sl = l; sl < kFwN; sl += kWave) {
                u64 key = L.tb_key[sl];
                if ((u32)(key >> 32) != rstamp) continue;
                u32 node = (u32)key;
                u32 x = L.tb_lvl[sl];
                S.R[2 * (int64_t)node] = (u64)P.tag | ((u64)(x & 0xFFFFu) << 32);
                S.R[2 * (int64_t)node + 1] = L.tb_acc[sl];
            }
        }
        __syncthreads();
        ac = blo + cut;
    }
}

// ------------------------------------------------------------ the kernel

__device__ void resolve_pair(const LaunchArgs &a, int64_t slot, Pair &P) {
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
    int64_t i = q - R.qoff;
    if (a.ps) {
        P.g = a.pg ? a.pg[q] : 0;
        P.s = a.ps[q];
        P.z = a.pz[q];
    } else {
        int64_t idx;
        if (R.graph >= 0) { P.g = R.graph; idx = R.base + i; }
        else { P.g = (int32_t)(i / R.per_graph); idx = R.base + (i % R.per_graph); }
        int32_t noff = a.g.seg_noff[P.g];
        int32_t ng = a.g.seg_noff[P.g + 1] - noff;
        u64 st = (u64)R.stream + (u64)STREAMS_PER_GRAPH * (u64)P.g;
        u64 s = __umul64hi(rng_word(R.seed, st, (u64)idx, 0), (u64)ng);
        u64 zp = __umul64hi(rng_word(R.seed, st, (u64)idx, 1), (u64)(ng - 1));
        P.s = (int32_t)s;
        P.z = (int32_t)(zp + (zp >= s ? 1 : 0));
        if (R.c > 0) P.lam = rng_word(R.seed, (u64)STREAM_RADE + (u64)STREAMS_PER_GRAPH * (u64)P.g, (u64)idx, 0);
    }
    P.noff = a.g.seg_noff[P.g];
    P.ng = a.g.seg_noff[P.g + 1] - P.noff;
    P.elo = a.g.seg_eoff[P.g];
    P.ehi = a.g.seg_eoff[P.g + 1];
    P.level = (P.opt == OPT_SH || P.opt == OPT_SFM);
}

__global__ void __launch_bounds__(64) k_sweep(LaunchArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int l = lane_id();
    const int64_t slab = blockIdx.x;
    Slab S;
    S.F = a.sl.F + slab * a.sl.nmax * 2;
    S.R = a.sl.R + slab * a.sl.nmax * 2;
    S.N = a.sl.N + slab * a.sl.nmax;
    S.AG = a.sl.AG + slab * a.sl.nmax * 2;
    S.AGF = a.sl.AGF + slab * a.sl.nmax;
    S.touched = a.sl.touched + slab * a.sl.nmax;
    S.arcs = a.sl.arcs + slab * a.sl.cap * 2;
    S.XS = a.sl.XS + slab * a.sl.gmax * 2;
    S.hdr = a.sl.hdr + slab * 4;
    TabLds &tab = *reinterpret_cast<TabLds *>(lds_raw);
    u32 *bm = reinterpret_cast<u32 *>(lds_raw + sizeof(TabLds));
    const int64_t bmw = a.lds_bitmap ? (a.sl.nmax + 31) / 32 : 0;
    // stamped tables start empty
    for (int i = l; i < kFwN; i += kWave) { tab.f.fw_key[i] = 0; }
    u32 serial = S.hdr[0];
    u32 agstamp = S.hdr[1];
    u32 stamp = 1;  // one counter for both table uses (they share LDS)
    __syncthreads();
    for (;;) {
        u32 qq = 0;
        if (l == 0) qq = atomicAdd(a.work, 1u);
        int64_t q = (int64_t)(u32)uni((int)qq);
        if (q >= a.npairs) break;
        Pair P;
        resolve_pair(a, q, P);
        serial += 1;
        if (serial == 0) serial = 1;  // tag 0 never valid (fresh slabs are zero)
        P.tag = serial;
        // window: first departure of s, last arrival at z, inside [t0, t1]
        const int32_t gs_node = P.noff + P.s, gz_node = P.noff + P.z;
        int64_t o0 = a.g.out_off[gs_node], o1 = a.g.out_off[gs_node + 1];
        int64_t i0 = a.g.in_off[gz_node], i1 = a.g.in_off[gz_node + 1];
        int64_t od = wave_lower_bound(a.g.out_t, o0, o1, P.t0);
        int64_t id = wave_upper_bound(a.g.in_t, i0, i1, P.t1) - 1;
        bool ok = od < o1 && id >= i0;
        int32_t dep = ok ? a.g.out_t[od] : 0, lin = ok ? a.g.in_t[id] : 0;
        ok = ok && dep <= P.t1 && lin >= P.t0 && lin >= dep;
        FwdOut fo;
        fo.reached = false; fo.zh = kHInf; fo.zS = 0; fo.t_arr = -1; fo.arcs = 0; fo.swept = 0; fo.flags = 0;
        if (ok) {
            P.lo = wave_lower_bound(a.g.T, P.elo, P.ehi, dep);
            P.hi = wave_upper_bound(a.g.T, P.lo, P.ehi, lin);
            // reset the reached bitmap, seed the origin
            for (int64_t w = l; w < bmw; w += kWave) bm[w] = 0;
            __syncthreads();
            if (l == 0) {
                S.F[2 * (int64_t)P.s] = (u64)P.tag;  // h = 0
                S.F[2 * (int64_t)P.s + 1] = 1ull;
                if (a.lds_bitmap) bm[P.s >> 5] |= 1u << (P.s & 31);
            }
            __syncthreads();
            forward(a, P, S, bm, tab.f, stamp, agstamp, fo);
            __syncthreads();
        }
        u32 flags = fo.flags;
        bool reach = ok && fo.reached && !(flags & (REC_HOPS_LIMIT | REC_ARCS_LIMIT));
        u64 sigma = reach ? fo.zS : 0;
        if (reach && sigma == kUMax) flags |= REC_OVERFLOW;
        bool do_rev = reach && !(flags & REC_OVERFLOW);
        RevCtx X;
        X.sigma = sigma; X.dsh = fo.zh; X.touched_n = 0; X.ovf = false;
        if (do_rev) {
            reverse(a, P, S, tab.r, stamp, fo.arcs, X);
            __syncthreads();
            // flow conservation at the origin: B(origin) must equal sigma
            u64 th = ld_agent(&S.R[2 * (int64_t)P.s]);
            u64 bo = 0;
            if ((u32)th == P.tag && (!P.level || ((u32)(th >> 32) & 0xFFFFu) == 0u)) bo = ld_agent(&S.R[2 * (int64_t)P.s + 1]);
            if (bo != sigma) flags |= REC_SELFCHECK;
        }
        if (X.ovf) flags |= REC_OVERFLOW;
        // finalize: f(v) = N(v) / sigma into the sums; reset N
        bool accum = do_rev && !(flags & REC_OVERFLOW);
        const DevReq *R = P.req;
        for (int64_t i = l; i < X.touched_n; i += kWave) {
            int32_t v = S.touched[i];
            u64 nv = atomicExch((unsigned long long *)&S.N[v], 0ull);
            if (!accum) continue;
            double f = (double)nv / (double)sigma;
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
        if (l == 0) {
            if (a.rec) {
                int32_t *rr = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(a.rec) + P.qout * 24);
                bool rch = reach;
                rr[0] = rch ? 1 : 0;
                rr[1] = rch ? fo.t_arr : -1;
                rr[2] = rch ? (int32_t)fo.zh : -1;
                rr[3] = (int32_t)flags;
                *reinterpret_cast<u64 *>(rr + 4) = sigma;
            }
            if (!(flags & REC_ARCS_LIMIT)) {
                atomicAdd((unsigned long long *)&a.stats[0], (unsigned long long)fo.swept);
                atomicAdd((unsigned long long *)&a.stats[1], (unsigned long long)fo.arcs);
            }
            if (flags & REC_OVERFLOW) atomicAdd((unsigned long long *)&a.stats[2], 1ull);
            if (reach) atomicAdd((unsigned long long *)&a.stats[3], 1ull);
            if (flags & REC_HOPS_LIMIT) atomicAdd((unsigned long long *)&a.stats[4], 1ull);
            if (flags & REC_SELFCHECK) atomicAdd((unsigned long long *)&a.stats[6], 1ull);
            if (flags & REC_ARCS_LIMIT) {
                atomicAdd((unsigned long long *)&a.stats[5], 1ull);
                int pos = atomicAdd(&a.retry[0], 1);
                a.retry[1 + pos] = (int32_t)P.q;
            }
        }
        __syncthreads();
    }
    if (l == 0) { S.hdr[0] = serial; S.hdr[1] = agstamp; }
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

__global__ void k_fill_u64(u64 *p, u64 val, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = val;
}

}  // namespace mantra

// ------------------------------------------------------------ launchers

extern "C" {
hipError_t mantra_launch_sweep(const mantra::LaunchArgs *a, int nslabs, size_t lds_bytes, hipStream_t st) {
    hipLaunchKernelGGL(mantra::k_sweep, dim3(nslabs), dim3(64), lds_bytes, st, *a);
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
size_t mantra_tab_lds_bytes(void) { return sizeof(mantra::TabLds); }
}
