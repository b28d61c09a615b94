/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY (the oracle).
 *
 * A plain, slow CPU statement of what MANTRA's per-sampled-pair hot path
 * computes.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may call it; the product library never links, loads or
 * executes anything here, and this file shares no code with it.
 *
 * What it computes, per ordered pair (s, z) of distinct nodes inside a time
 * window [t0, t1] (Preliminaries, "Temporal Graphs, and Paths", Definition 1,
 * "Temporal Betweenness Centrality"; Appendix A for temporal edges):
 *
 *   * a temporal walk is a sequence of temporal edges (v_{i-1}, v_i, t_i) with
 *     v_0 = s and strictly increasing times; s starts at the origin
 *     appearance (s, -inf), which precedes every edge;
 *   * the appearance DAG has one node per vertex appearance (v, t) (an edge
 *     into v at time t) plus the origin, and one arc (u,t') -> (v,t) per edge
 *     (u, v, t) and per appearance (u, t') of its tail with t' < t;  walks
 *     from s are exactly the origin-rooted paths of this DAG;
 *   * sh  : walks with the minimum number of hops to z;
 *     sfm : walks that arrive at the earliest arrival time t*(z) and, among
 *           those, have the minimum number of hops;
 *     pfm : walks whose every prefix ending at v_i arrives at t*(v_i);
 *     fm  : every walk arriving at t*(z) (walks, not simple paths: counting
 *           foremost simple paths is #P-hard, walks are countable; a visit of
 *           v is counted with multiplicity);
 *   * sigma = number of optimal walks; N(v) = number of (optimal walk,
 *     internal visit of v) pairs for v not in {s, z}; N(e) = number of
 *     optimal walks using temporal edge e (first and last edges included);
 *     f(v|s,z) = N(v)/sigma and f(e|s,z) = N(e)/sigma (the estimator of
 *     Section 4.1), 0 when z is unreachable.
 *
 * Counts are uint64 and saturate at 2^64-1: saturating + and x of
 * non-negative integers give min(true value, 2^64-1) exactly, so a
 * saturated count never rounds and is comparable bit for bit.
 *
 * Two modes compute the same sums:
 *   mode 0 ("explicit"): every arc is enumerated, forward and backward;
 *   mode 1 ("prefix")  : the sum over the tail appearances of u older than t
 *                        is read from running per-node aggregates of the
 *                        finished appearances of u (same sums, fewer loops),
 *                        for windows too large for mode 0.
 * The tests cross-check both modes against each other and mode 0 against a
 * brute-force enumeration of walks.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <limits.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define U64MAX 0xFFFFFFFFFFFFFFFFull
#define DINF INT32_MAX

enum { OPT_SH = 0, OPT_FM = 1, OPT_SFM = 2, OPT_PFM = 3 };
enum { REC_OVERFLOW = 1, REC_SELFCHECK = 2 };

static inline uint64_t sadd(uint64_t a, uint64_t b) { uint64_t c = a + b; return c < a ? U64MAX : c; }
static inline uint64_t smul(uint64_t a, uint64_t b) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    return p > (unsigned __int128)U64MAX ? U64MAX : (uint64_t)p;
}

typedef struct {
    int32_t reachable;
    int32_t t_arr;  /* earliest arrival among the optimal walks, -1 if unreachable */
    int32_t hops;   /* fewest hops among the optimal walks, -1 if unreachable */
    int32_t flags;  /* REC_OVERFLOW: sigma (or an fm N(v)) saturated */
    uint64_t sigma;
} orc_record;

typedef struct {
    int32_t n;
    int64_t m;
    int32_t *src, *dst, *t;
    int64_t *ord;  /* edge ids sorted by (t, id) */
    int32_t *ts;   /* t[ord[k]] */
} orc_graph;

/* ------------------------------------------------------------------------ */
/* counter-based random numbers: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) */

#define SM_GAMMA 0x9E3779B97F4A7C15ull
static inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
/* k-th output (k >= 1) of a SplitMix64 generator started at state x */
uint64_t orc_splitmix_nth(uint64_t x, uint64_t k) { return sm_mix(x + k * SM_GAMMA); }
/* word j (0..3) of draw i on a stream: the (4i+j+1)-th output of SplitMix64
   started at key = the (stream+1)-th output of SplitMix64 started at seed */
uint64_t orc_word(uint64_t seed, uint64_t stream, uint64_t i, uint64_t j) {
    uint64_t key = orc_splitmix_nth(seed, stream + 1);
    return orc_splitmix_nth(key, 4 * i + j + 1);
}
static inline uint64_t mulhi(uint64_t x, uint64_t n) {
    return (uint64_t)(((unsigned __int128)x * (unsigned __int128)n) >> 64);
}
/* pairs i0..i0+k-1 of a stream: uniform over ordered pairs s != z */
void orc_draw_pairs(uint64_t seed, uint64_t stream, int32_t n, int64_t i0, int64_t k,
                    int32_t *S, int32_t *Z) {
    for (int64_t q = 0; q < k; ++q) {
        uint64_t i = (uint64_t)(i0 + q);
        uint64_t s = mulhi(orc_word(seed, stream, i, 0), (uint64_t)n);
        uint64_t zp = mulhi(orc_word(seed, stream, i, 1), (uint64_t)(n - 1));
        S[q] = (int32_t)s;
        Z[q] = (int32_t)(zp + (zp >= s ? 1 : 0));
    }
}

/* ------------------------------------------------------------------------ */
/* graph */

static const int32_t *g_sort_t;
static int cmp_edge(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    int32_t tx = g_sort_t[x], ty = g_sort_t[y];
    if (tx != ty) return tx < ty ? -1 : 1;
    return x < y ? -1 : (x > y);
}

orc_graph *orc_graph_new(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                         const int32_t *t) {
    orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
    g->n = n;
    g->m = m;
    g->src = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    g->dst = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    g->t = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    g->ord = (int64_t *)malloc(sizeof(int64_t) * (m ? m : 1));
    g->ts = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    memcpy(g->src, src, sizeof(int32_t) * m);
    memcpy(g->dst, dst, sizeof(int32_t) * m);
    memcpy(g->t, t, sizeof(int32_t) * m);
    for (int64_t i = 0; i < m; ++i) g->ord[i] = i;
    g_sort_t = g->t; /* not re-entrant: graphs are built one at a time */
    qsort(g->ord, (size_t)m, sizeof(int64_t), cmp_edge);
    for (int64_t k = 0; k < m; ++k) g->ts[k] = g->t[g->ord[k]];
    return g;
}

void orc_graph_free(orc_graph *g) {
    if (!g) return;
    free(g->src); free(g->dst); free(g->t); free(g->ord); free(g->ts);
    free(g);
}

/* ------------------------------------------------------------------------ */
/* per-pair workspace: window edges, appearances, out-lists */

typedef struct {
    int64_t W, A;
    int32_t *wu, *wv, *wt;   /* window edges in time order */
    int64_t *wid;            /* their original edge ids */
    int64_t *head;           /* window edge -> head appearance */
    int64_t *app_off;        /* [n+1] appearances grouped by node, ascending time */
    int32_t *app_time, *app_node;
    int64_t *app_order;      /* appearance ids in ascending time */
    int64_t *out_off, *out_k;/* window edges grouped by tail, ascending time */
    uint8_t *reach, *term;
    int32_t *dist, *hopP, *tstar;
    int64_t *first_app;      /* [n] first reached appearance of v, -1 if none */
    uint64_t *sigT, *sigW, *sigP, *B, *tailagg, *tailP;
} pws;

static void pws_free(pws *w) {
    free(w->wu); free(w->wv); free(w->wt); free(w->wid); free(w->head);
    free(w->app_off); free(w->app_time); free(w->app_node); free(w->app_order);
    free(w->out_off); free(w->out_k); free(w->reach); free(w->term); free(w->dist);
    free(w->hopP); free(w->tstar); free(w->first_app); free(w->sigT); free(w->sigW);
    free(w->sigP); free(w->B); free(w->tailagg); free(w->tailP);
}

static int64_t lower_ts(const orc_graph *g, int32_t x) { /* first k with ts[k] >= x */
    int64_t lo = 0, hi = g->m;
    while (lo < hi) { int64_t md = (lo + hi) / 2; if (g->ts[md] < x) lo = md + 1; else hi = md; }
    return lo;
}

static void pws_build(const orc_graph *g, int32_t t0, int32_t t1, pws *w) {
    int32_t n = g->n;
    int64_t lo = lower_ts(g, t0);
    int64_t hi = (t1 == INT32_MAX) ? g->m : lower_ts(g, t1 + 1);
    if (hi < lo) hi = lo;
    int64_t W = hi - lo;
    w->W = W;
    size_t Wa = (size_t)(W ? W : 1);
    w->wu = (int32_t *)malloc(sizeof(int32_t) * Wa);
    w->wv = (int32_t *)malloc(sizeof(int32_t) * Wa);
    w->wt = (int32_t *)malloc(sizeof(int32_t) * Wa);
    w->wid = (int64_t *)malloc(sizeof(int64_t) * Wa);
    w->head = (int64_t *)malloc(sizeof(int64_t) * Wa);
    for (int64_t k = 0; k < W; ++k) {
        int64_t e = g->ord[lo + k];
        w->wid[k] = e; w->wu[k] = g->src[e]; w->wv[k] = g->dst[e]; w->wt[k] = g->t[e];
    }
    /* appearances: distinct (v, t) heads */
    int32_t *last = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) last[v] = INT32_MIN;
    w->app_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t A = 0;
    for (int64_t k = 0; k < W; ++k) {
        int32_t v = w->wv[k];
        if (last[v] != w->wt[k]) { last[v] = w->wt[k]; w->app_off[v + 1]++; A++; }
    }
    for (int32_t v = 0; v < n; ++v) w->app_off[v + 1] += w->app_off[v];
    w->A = A;
    size_t Aa = (size_t)(A ? A : 1);
    w->app_time = (int32_t *)malloc(sizeof(int32_t) * Aa);
    w->app_node = (int32_t *)malloc(sizeof(int32_t) * Aa);
    w->app_order = (int64_t *)malloc(sizeof(int64_t) * Aa);
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) { cur[v] = w->app_off[v]; last[v] = INT32_MIN; }
    int64_t na = 0;
    for (int64_t k = 0; k < W; ++k) {
        int32_t v = w->wv[k];
        if (last[v] != w->wt[k]) {
            last[v] = w->wt[k];
            int64_t a = cur[v]++;
            w->app_time[a] = w->wt[k];
            w->app_node[a] = v;
            w->app_order[na++] = a;
        }
        w->head[k] = cur[v] - 1;
    }
    /* out-lists by tail */
    w->out_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    w->out_k = (int64_t *)malloc(sizeof(int64_t) * Wa);
    for (int64_t k = 0; k < W; ++k) w->out_off[w->wu[k] + 1]++;
    for (int32_t v = 0; v < n; ++v) w->out_off[v + 1] += w->out_off[v];
    for (int32_t v = 0; v < n; ++v) cur[v] = w->out_off[v];
    for (int64_t k = 0; k < W; ++k) w->out_k[cur[w->wu[k]]++] = k;
    free(cur);
    free(last);
    w->reach = (uint8_t *)calloc(Aa, 1);
    w->term = (uint8_t *)calloc(Aa, 1);
    w->dist = (int32_t *)malloc(sizeof(int32_t) * Aa);
    w->hopP = (int32_t *)malloc(sizeof(int32_t) * Aa);
    for (int64_t a = 0; a < A; ++a) { w->dist[a] = DINF; w->hopP[a] = DINF; }
    w->sigT = (uint64_t *)calloc(Aa, sizeof(uint64_t));
    w->sigW = (uint64_t *)calloc(Aa, sizeof(uint64_t));
    w->sigP = (uint64_t *)calloc(Aa, sizeof(uint64_t));
    w->B = (uint64_t *)calloc(Aa, sizeof(uint64_t));
    w->tailagg = (uint64_t *)calloc(Wa, sizeof(uint64_t));
    w->tailP = (uint64_t *)calloc(Wa, sizeof(uint64_t));
    w->tstar = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    w->first_app = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
}

/* min-hop relaxation of appearance a by a tail of hop count db and count sb */
static inline void relax(pws *w, int64_t a, int32_t db, uint64_t sb) {
    int32_t d = db + 1;
    if (d < w->dist[a]) { w->dist[a] = d; w->sigT[a] = sb; }
    else if (d == w->dist[a]) w->sigT[a] = sadd(w->sigT[a], sb);
}

/* forward pass over all arcs, enumerated one by one */
static void forward_explicit(pws *w, int32_t s) {
    for (int64_t k = 0; k < w->W; ++k) {
        int32_t u = w->wu[k], t = w->wt[k];
        int64_t a = w->head[k];
        if (u == s) { /* arc from the origin (s, -inf) */
            w->reach[a] = 1;
            relax(w, a, 0, 1);
            w->sigW[a] = sadd(w->sigW[a], 1);
        }
        for (int64_t b = w->app_off[u]; b < w->app_off[u + 1] && w->app_time[b] < t; ++b) {
            if (!w->reach[b]) continue;
            w->reach[a] = 1;
            relax(w, a, w->dist[b], w->sigT[b]);
            w->sigW[a] = sadd(w->sigW[a], w->sigW[b]);
        }
    }
}

/* forward pass reading the finished appearances of each tail through running
   per-node aggregates: minimum hop count, count at that minimum, walk total */
static void forward_prefix(pws *w, int32_t n, int32_t s, int32_t opt) {
    int32_t *mn = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint64_t *sm = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    uint64_t *wc = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    for (int32_t v = 0; v < n; ++v) mn[v] = DINF;
    int64_t k = 0, ap = 0;
    while (k < w->W) {
        int32_t t = w->wt[k];
        int64_t k1 = k;
        while (k1 < w->W && w->wt[k1] == t) ++k1;
        for (int64_t q = k; q < k1; ++q) {
            int32_t u = w->wu[q];
            int64_t a = w->head[q];
            if (u == s) { w->reach[a] = 1; relax(w, a, 0, 1); w->sigW[a] = sadd(w->sigW[a], 1); }
            if (mn[u] != DINF) { w->reach[a] = 1; relax(w, a, mn[u], sm[u]); }
            if (wc[u]) w->sigW[a] = sadd(w->sigW[a], wc[u]);
        }
        /* counted-tail sums of the edges at time t (the heads are final now,
           the tails' aggregates still cover only appearances older than t) */
        for (int64_t q = k; q < k1; ++q) {
            int32_t u = w->wu[q];
            int64_t h = w->head[q];
            if (opt == OPT_FM) {
                w->tailagg[q] = sadd(u == s ? 1 : 0, wc[u]);
            } else if (opt == OPT_SH || opt == OPT_SFM) {
                uint64_t x = (u == s && w->dist[h] == 1) ? 1 : 0;
                if (mn[u] != DINF && mn[u] + 1 == w->dist[h]) x = sadd(x, sm[u]);
                w->tailagg[q] = x;
            }
        }
        /* the appearances created at time t are finished: fold them in */
        while (ap < w->A && w->app_time[w->app_order[ap]] == t) {
            int64_t a = w->app_order[ap++];
            int32_t v = w->app_node[a];
            if (!w->reach[a]) continue;
            wc[v] = sadd(wc[v], w->sigW[a]);
            if (w->dist[a] < mn[v]) { mn[v] = w->dist[a]; sm[v] = w->sigT[a]; }
            else if (w->dist[a] == mn[v]) sm[v] = sadd(sm[v], w->sigT[a]);
        }
        k = k1;
    }
    free(mn); free(sm); free(wc);
}

static void earliest(pws *w, int32_t n) {
    for (int32_t v = 0; v < n; ++v) {
        w->tstar[v] = DINF;
        w->first_app[v] = -1;
        for (int64_t a = w->app_off[v]; a < w->app_off[v + 1]; ++a)
            if (w->reach[a]) { w->tstar[v] = w->app_time[a]; w->first_app[v] = a; break; }
    }
}

/* pfm counts: only the appearance (v, t*(v)) of each v, fed by the
   appearance (u, t*(u)) of each tail with t*(u) < t */
static void forward_pfm(pws *w, int32_t s) {
    for (int64_t k = 0; k < w->W; ++k) {
        int32_t u = w->wu[k], v = w->wv[k], t = w->wt[k];
        if (v == s || t != w->tstar[v]) continue;
        int64_t a = w->head[k];
        if (u == s) {
            w->sigP[a] = sadd(w->sigP[a], 1);
            if (1 < w->hopP[a]) w->hopP[a] = 1;
            w->tailP[k] = 1;
        } else if (w->tstar[u] < t) {
            int64_t b = w->first_app[u];
            w->sigP[a] = sadd(w->sigP[a], w->sigP[b]);
            if (w->hopP[b] + 1 < w->hopP[a]) w->hopP[a] = w->hopP[b] + 1;
            w->tailP[k] = w->sigP[b];
        }
    }
}

static inline int pfm_app(const pws *w, int64_t a, int32_t s) {
    int32_t v = w->app_node[a];
    return v != s && w->first_app[v] == a;
}

/* is arc tail-appearance a (-1 = origin) -> head appearance h counted? */
static inline int arc_counted(const pws *w, int32_t opt, int32_t s, int64_t a, int64_t h) {
    if (opt == OPT_FM) return a < 0 ? 1 : w->reach[a];
    if (opt == OPT_PFM) {
        if (!pfm_app(w, h, s)) return 0;
        return a < 0 ? 1 : pfm_app(w, a, s);
    }
    if (a < 0) return w->dist[h] == 1;
    return w->reach[a] && w->dist[a] + 1 == w->dist[h];
}

static inline uint64_t app_sig(const pws *w, int32_t opt, int32_t s, int64_t a) {
    if (opt == OPT_FM) return w->reach[a] ? w->sigW[a] : 0;
    if (opt == OPT_PFM) return pfm_app(w, a, s) ? w->sigP[a] : 0;
    return w->reach[a] ? w->sigT[a] : 0;
}

/* backward pass: B(a) = number of counted continuations a -> terminal */
static uint64_t backward_explicit(pws *w, int32_t opt, int32_t s) {
    for (int64_t q = w->A - 1; q >= 0; --q) {
        int64_t a = w->app_order[q];
        if (w->term[a]) { w->B[a] = 1; continue; }
        if (opt == OPT_PFM ? !pfm_app(w, a, s) : !w->reach[a]) continue;
        int32_t v = w->app_node[a], ta = w->app_time[a];
        uint64_t b = 0;
        for (int64_t j = w->out_off[v]; j < w->out_off[v + 1]; ++j) {
            int64_t k = w->out_k[j];
            if (w->wt[k] <= ta) continue;
            int64_t h = w->head[k];
            if (arc_counted(w, opt, s, a, h)) b = sadd(b, w->B[h]);
        }
        w->B[a] = b;
    }
    uint64_t bo = 0; /* origin */
    for (int64_t j = w->out_off[s]; j < w->out_off[s + 1]; ++j) {
        int64_t h = w->head[w->out_k[j]];
        if (arc_counted(w, opt, s, -1, h)) bo = sadd(bo, w->B[h]);
    }
    return bo;
}

/* open-addressing map (node, level) -> running sum, for mode 1 sh/sfm */
typedef struct { uint64_t *key; uint64_t *val; uint64_t cap; } lmap;
static void lmap_init(lmap *m, int64_t want) {
    uint64_t c = 16;
    while (c < (uint64_t)(2 * want + 16)) c <<= 1;
    m->cap = c;
    m->key = (uint64_t *)malloc(sizeof(uint64_t) * c);
    m->val = (uint64_t *)calloc(c, sizeof(uint64_t));
    for (uint64_t i = 0; i < c; ++i) m->key[i] = U64MAX;
}
static uint64_t *lmap_slot(lmap *m, uint64_t k, int create) {
    uint64_t i = sm_mix(k) & (m->cap - 1);
    while (m->key[i] != U64MAX) {
        if (m->key[i] == k) return &m->val[i];
        i = (i + 1) & (m->cap - 1);
    }
    if (!create) return NULL;
    m->key[i] = k;
    return &m->val[i];
}

static uint64_t backward_prefix(pws *w, int32_t opt, int32_t n, int32_t s) {
    uint64_t *run = NULL;
    lmap mp = {0};
    int lev = (opt == OPT_SH || opt == OPT_SFM);
    if (lev) lmap_init(&mp, w->W);
    else run = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    int64_t k = w->W - 1, ap = w->A - 1;
    while (k >= 0) {
        int32_t t = w->wt[k];
        /* appearances at time t read sums over out-arcs later than t */
        while (ap >= 0 && w->app_time[w->app_order[ap]] == t) {
            int64_t a = w->app_order[ap--];
            int32_t v = w->app_node[a];
            if (w->term[a]) { w->B[a] = 1; continue; }
            if (opt == OPT_PFM ? !pfm_app(w, a, s) : !w->reach[a]) continue;
            if (lev) {
                uint64_t *p = lmap_slot(&mp, ((uint64_t)v << 32) | (uint32_t)w->dist[a], 0);
                w->B[a] = p ? *p : 0;
            } else {
                w->B[a] = run[v];
            }
        }
        /* then the edges at time t feed their tails */
        for (; k >= 0 && w->wt[k] == t; --k) {
            int64_t h = w->head[k];
            int32_t u = w->wu[k];
            if (!w->B[h]) continue;
            if (lev) {
                if (!w->reach[h]) continue;
                uint64_t *p = lmap_slot(&mp, ((uint64_t)u << 32) | (uint32_t)(w->dist[h] - 1), 1);
                *p = sadd(*p, w->B[h]);
            } else if (opt == OPT_PFM) {
                if (pfm_app(w, h, s)) run[u] = sadd(run[u], w->B[h]);
            } else {
                run[u] = sadd(run[u], w->B[h]);
            }
        }
    }
    uint64_t bo;
    if (lev) { uint64_t *p = lmap_slot(&mp, ((uint64_t)s << 32) | 0u, 0); bo = p ? *p : 0; }
    else bo = run[s];
    if (lev) { free(mp.key); free(mp.val); } else free(run);
    return bo;
}

/* counted-tail sum of a window edge k (sum of sigma over the tail
   appearances, origin included, whose arc into head(k) is counted) */
static uint64_t tail_sum_explicit(const pws *w, int32_t opt, int32_t s, int64_t k) {
    int32_t u = w->wu[k], t = w->wt[k];
    int64_t h = w->head[k];
    uint64_t acc = 0;
    if (u == s && arc_counted(w, opt, s, -1, h)) acc = 1;
    for (int64_t b = w->app_off[u]; b < w->app_off[u + 1] && w->app_time[b] < t; ++b)
        if (arc_counted(w, opt, s, b, h)) acc = sadd(acc, app_sig(w, opt, s, b));
    return acc;
}

/*
 * One pair.  nodeN [n] and edgeN [m] (original edge ids) are optional dense
 * outputs, zero-filled here.  Returns 0, or -1 on bad arguments.
 */
int orc_pair(const orc_graph *g, int32_t opt, int32_t t0, int32_t t1, int32_t s, int32_t z,
             int32_t mode, orc_record *rec, uint64_t *nodeN, uint64_t *edgeN) {
    int32_t n = g->n;
    if (s < 0 || s >= n || z < 0 || z >= n || s == z || opt < 0 || opt > 3) return -1;
    if (nodeN) memset(nodeN, 0, sizeof(uint64_t) * (size_t)n);
    if (edgeN) memset(edgeN, 0, sizeof(uint64_t) * (size_t)g->m);
    pws w;
    memset(&w, 0, sizeof(w));
    pws_build(g, t0, t1, &w);
    if (mode == 0) forward_explicit(&w, s); else forward_prefix(&w, n, s, opt);
    earliest(&w, n);
    forward_pfm(&w, s);
    rec->reachable = 0; rec->t_arr = -1; rec->hops = -1; rec->flags = 0; rec->sigma = 0;
    if (w.first_app[z] < 0) { pws_free(&w); return 0; }
    uint64_t sigma = 0;
    if (opt == OPT_SH) {
        int32_t d = DINF;
        for (int64_t a = w.app_off[z]; a < w.app_off[z + 1]; ++a)
            if (w.reach[a] && w.dist[a] < d) d = w.dist[a];
        int32_t ta = DINF;
        for (int64_t a = w.app_off[z]; a < w.app_off[z + 1]; ++a)
            if (w.reach[a] && w.dist[a] == d) {
                w.term[a] = 1;
                sigma = sadd(sigma, w.sigT[a]);
                if (w.app_time[a] < ta) ta = w.app_time[a];
            }
        rec->t_arr = ta; rec->hops = d;
    } else {
        int64_t a = w.first_app[z];
        w.term[a] = 1;
        rec->t_arr = w.app_time[a];
        if (opt == OPT_FM) { sigma = w.sigW[a]; rec->hops = w.dist[a]; }
        else if (opt == OPT_SFM) { sigma = w.sigT[a]; rec->hops = w.dist[a]; }
        else { sigma = w.sigP[a]; rec->hops = w.hopP[a]; }
    }
    rec->reachable = 1;
    rec->sigma = sigma;
    uint64_t bo = (mode == 0) ? backward_explicit(&w, opt, s) : backward_prefix(&w, opt, n, s);
    if (bo != sigma) rec->flags |= REC_SELFCHECK; /* flow conservation at the origin */
    if (sigma == U64MAX) rec->flags |= REC_OVERFLOW;
    /* node dependencies: sum over the appearances of v of sigma(a) * B(a) */
    for (int32_t v = 0; v < n; ++v) {
        if (v == s || v == z) continue;
        uint64_t acc = 0;
        for (int64_t a = w.app_off[v]; a < w.app_off[v + 1]; ++a)
            if (w.B[a]) acc = sadd(acc, smul(app_sig(&w, opt, s, a), w.B[a]));
        if (opt == OPT_FM && acc == U64MAX) rec->flags |= REC_OVERFLOW;
        if (nodeN) nodeN[v] = acc;
    }
    /* edge dependencies: counted-tail sum times B(head) */
    if (edgeN) {
        for (int64_t k = 0; k < w.W; ++k) {
            int64_t h = w.head[k];
            if (!w.B[h]) continue;
            uint64_t ts;
            if (mode == 0) ts = tail_sum_explicit(&w, opt, s, k);
            else ts = (opt == OPT_PFM) ? (pfm_app(&w, h, s) ? w.tailP[k] : 0) : w.tailagg[k];
            edgeN[w.wid[k]] = smul(ts, w.B[h]);
        }
    }
    pws_free(&w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* sums over a list of pairs: the estimator's running sums of Algorithm 1     */

typedef struct { double hi, lo; } dd;
static inline void dd_add(double *hi, double *lo, double x) { /* Neumaier two-sum */
    double s = *hi + x;
    double bp = s - *hi;
    double e = (*hi - (s - bp)) + (x - bp);
    *hi = s;
    *lo += e;
}

typedef struct {
    int64_t nn, ne;
    int32_t *node; double *fn;
    int64_t *edge; double *fe;
} sparse_out;

/*
 * For pairs q = 0..np-1 (S[q], Z[q]) add f, f^2 and lambda_j f (j < c, lambda
 * from bit j of lam[q]: +1 if the bit is 0, -1 if it is 1) into double-double
 * accumulators, and f(e) into the edge accumulators if ehi != NULL.  Pairs are
 * evaluated in parallel and added in pair order.  recs[np] receives the
 * per-pair records.  Returns the number of pairs whose counts saturated.
 */
int64_t orc_accumulate(const orc_graph *g, int32_t opt, int32_t t0, int32_t t1, int32_t mode,
                       int64_t np, const int32_t *S, const int32_t *Z, int32_t c,
                       const uint64_t *lam, double *bhi, double *blo, double *whi, double *wlo,
                       double *rhi, double *rlo, double *ehi, double *elo, orc_record *recs,
                       int32_t nthreads) {
    int32_t n = g->n;
    int64_t noverflow = 0;
    const int64_t batch = 256;
    sparse_out *outs = (sparse_out *)calloc((size_t)batch, sizeof(sparse_out));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    for (int64_t q0 = 0; q0 < np; q0 += batch) {
        int64_t q1 = q0 + batch < np ? q0 + batch : np;
#pragma omp parallel
        {
            uint64_t *nN = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
            uint64_t *eN = ehi ? (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(g->m ? g->m : 1)) : NULL;
#pragma omp for schedule(dynamic, 1)
            for (int64_t q = q0; q < q1; ++q) {
                sparse_out *o = &outs[q - q0];
                orc_pair(g, opt, t0, t1, S[q], Z[q], mode, &recs[q], nN, eN);
                o->nn = o->ne = 0;
                o->node = NULL; o->fn = NULL; o->edge = NULL; o->fe = NULL;
                orc_record *r = &recs[q];
                if (!r->reachable || (r->flags & REC_OVERFLOW)) continue;
                double sg = (double)r->sigma;
                int64_t cnt = 0;
                for (int32_t v = 0; v < n; ++v) cnt += nN[v] != 0;
                o->node = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt ? cnt : 1));
                o->fn = (double *)malloc(sizeof(double) * (size_t)(cnt ? cnt : 1));
                for (int32_t v = 0; v < n; ++v)
                    if (nN[v]) { o->node[o->nn] = v; o->fn[o->nn] = (double)nN[v] / sg; o->nn++; }
                if (eN) {
                    int64_t ce = 0;
                    for (int64_t e = 0; e < g->m; ++e) ce += eN[e] != 0;
                    o->edge = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ce ? ce : 1));
                    o->fe = (double *)malloc(sizeof(double) * (size_t)(ce ? ce : 1));
                    for (int64_t e = 0; e < g->m; ++e)
                        if (eN[e]) { o->edge[o->ne] = e; o->fe[o->ne] = (double)eN[e] / sg; o->ne++; }
                }
            }
            free(nN);
            free(eN);
        }
        for (int64_t q = q0; q < q1; ++q) {
            sparse_out *o = &outs[q - q0];
            if (recs[q].flags & REC_OVERFLOW) noverflow++;
            for (int64_t i = 0; i < o->nn; ++i) {
                int32_t v = o->node[i];
                double f = o->fn[i];
                double f2 = f * f;
                dd_add(&bhi[v], &blo[v], f);
                dd_add(&whi[v], &wlo[v], f2);
                for (int32_t j = 0; j < c; ++j) {
                    double x = ((lam[q] >> j) & 1) ? -f : f;
                    dd_add(&rhi[(int64_t)v * c + j], &rlo[(int64_t)v * c + j], x);
                }
            }
            for (int64_t i = 0; i < o->ne; ++i) dd_add(&ehi[o->edge[i]], &elo[o->edge[i]], o->fe[i]);
            free(o->node); free(o->fn); free(o->edge); free(o->fe);
        }
    }
    free(outs);
    return noverflow;
}

/* ------------------------------------------------------------------------ */
/* distances from single sources (the temporal BFS of Algorithm 2)           */

/*
 * For each source S[q] (q < k) and every node v: hops[q*n + v] = the hop
 * count of the record of the pair (S[q], v) -- the fewest hops over all walks
 * for sh, over the walks arriving first for sfm and fm, the hops of the
 * prefix-foremost walks for pfm -- or -1 where v is not reachable in the
 * window and for v = S[q].  The window starts at t0 for every source (the
 * pair record's window: a walk of s starts at its first departure >= t0).
 * Sources are evaluated in parallel.  Returns 0, or -1 on a bad argument.
 */
int orc_source_hops(const orc_graph *g, int32_t opt, int32_t t0, int32_t t1, int32_t mode, int64_t k,
                    const int32_t *S, int32_t *hops, int32_t nthreads) {
    int32_t n = g->n;
    if (opt < 0 || opt > 3) return -1;
    for (int64_t q = 0; q < k; ++q)
        if (S[q] < 0 || S[q] >= n) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < k; ++q) {
        int32_t s = S[q];
        int32_t *out = hops + q * (int64_t)n;
        pws w;
        memset(&w, 0, sizeof(w));
        pws_build(g, t0, t1, &w);
        if (mode == 0) forward_explicit(&w, s); else forward_prefix(&w, n, s, opt);
        earliest(&w, n);
        forward_pfm(&w, s);
        for (int32_t v = 0; v < n; ++v) {
            out[v] = -1;
            if (v == s || w.first_app[v] < 0) continue;
            if (opt == OPT_SH) {
                int32_t d = DINF;
                for (int64_t a = w.app_off[v]; a < w.app_off[v + 1]; ++a)
                    if (w.reach[a] && w.dist[a] < d) d = w.dist[a];
                out[v] = d;
            } else if (opt == OPT_PFM) {
                out[v] = w.hopP[w.first_app[v]];
            } else {
                out[v] = w.dist[w.first_app[v]];
            }
        }
        pws_free(&w);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* the TRK estimator's path sampler (appendix on other estimators)          */

/* draw j of pair i on a path stream: the SplitMix64 output (i * 2^16 + j + 1)
   of the generator started at the (2^20 + stream + 1)-th output of the one
   started at seed */
uint64_t orc_trk_word(uint64_t seed, uint64_t stream, uint64_t i, uint64_t j) {
    uint64_t key = orc_splitmix_nth(seed, ((uint64_t)1 << 20) + stream + 1);
    return orc_splitmix_nth(key, (i << 16) + j + 1);
}

typedef struct { int64_t k; uint64_t w; } trk_cand;
static const pws *g_trk_w;
static int cmp_trk(const void *a, const void *b) { /* (time, head, tail) ascending; origin (k < 0) first */
    int64_t x = ((const trk_cand *)a)->k, y = ((const trk_cand *)b)->k;
    if (x < 0 || y < 0) return (x < 0) ? (y < 0 ? 0 : -1) : 1;
    const pws *w = g_trk_w;
    if (w->wt[x] != w->wt[y]) return w->wt[x] < w->wt[y] ? -1 : 1;
    if (w->wv[x] != w->wv[y]) return w->wv[x] < w->wv[y] ? -1 : 1;
    return w->wu[x] < w->wu[y] ? -1 : (w->wu[x] > w->wu[y]);
}

/*
 * One optimal walk of the pair (s, z), drawn backwards with probability
 * 1/sigma_sz: the terminal appearance (z, t_z) with probability
 * sigma(z, t_z)/sigma_sz, then repeatedly a predecessor appearance (w, t_w)
 * of the current one with probability sigma(w, t_w)/sigma(current).  The
 * draws are arranged by edge: one draw picks an edge into the current
 * node's candidate appearances with probability (its counted-tail sum) /
 * (their total), which picks the appearance (with probability sigma(b) /
 * total) and the edge into it (with probability (tail sum) / sigma(b)) at
 * once.  Candidates are taken in the order (time, head id, tail id), the
 * origin first where it is one, and the draw r = floor(word * W / 2^64)
 * picks the first whose running total exceeds r.
 * rec gets the pair's record (as orc_pair); nodeV[v] the walk's internal
 * visits of v (v not s, z), edgeV[e] its uses of edge e (original ids).
 * Returns 0; -1 on bad arguments; -2 if a step's total disagrees with the
 * count it stands for or saturates (no walk then; the record is kept).
 */
int orc_trk_path(const orc_graph *g, int32_t opt, int32_t t0, int32_t t1, int32_t s, int32_t z, uint64_t seed,
                 uint64_t stream, uint64_t i, orc_record *rec, uint64_t *nodeV, uint64_t *edgeV) {
    int32_t n = g->n;
    int rc = orc_pair(g, opt, t0, t1, s, z, 0, rec, NULL, NULL);
    if (rc) return rc;
    /* the walk needs sigma only: the record's saturation flag is sigma's
       (orc_pair also flags an fm visit count N(v) that saturates) */
    rec->flags &= ~REC_OVERFLOW;
    if (rec->reachable && rec->sigma == U64MAX) rec->flags |= REC_OVERFLOW;
    if (nodeV) memset(nodeV, 0, sizeof(uint64_t) * (size_t)n);
    if (edgeV) memset(edgeV, 0, sizeof(uint64_t) * (size_t)g->m);
    if (!rec->reachable || (rec->flags & REC_OVERFLOW)) return 0;
    pws w;
    memset(&w, 0, sizeof(w));
    pws_build(g, t0, t1, &w);
    forward_explicit(&w, s);
    earliest(&w, n);
    forward_pfm(&w, s);
    /* terminal appearances of z */
    uint8_t *cand_app = (uint8_t *)calloc((size_t)(w.A ? w.A : 1), 1);
    if (opt == OPT_SH) {
        for (int64_t a = w.app_off[z]; a < w.app_off[z + 1]; ++a)
            if (w.reach[a] && w.dist[a] == rec->hops) cand_app[a] = 1;
    } else {
        cand_app[w.first_app[z]] = 1;
    }
    trk_cand *cs = (trk_cand *)malloc(sizeof(trk_cand) * (size_t)(w.W + 1));
    uint64_t expect = rec->sigma;
    int origin = 0;
    int ret = 0;
    for (uint64_t j = 0;; ++j) {
        /* candidates: edges into the candidate appearances, weighted by their
           counted-tail sums; the origin (weight 1) when it is one */
        int64_t nc = 0;
        if (origin) { cs[nc].k = -1; cs[nc].w = 1; nc++; }
        for (int64_t k = 0; k < w.W; ++k) {
            if (!cand_app[w.head[k]]) continue;
            uint64_t ts = tail_sum_explicit(&w, opt, s, k);
            if (ts) { cs[nc].k = k; cs[nc].w = ts; nc++; }
        }
        g_trk_w = &w; /* not re-entrant: walks are drawn one at a time */
        qsort(cs, (size_t)nc, sizeof(trk_cand), cmp_trk);
        uint64_t W = 0;
        for (int64_t c = 0; c < nc; ++c) W = sadd(W, cs[c].w);
        if (W != expect || W == 0 || W == U64MAX) { ret = -2; break; }
        uint64_t r = mulhi(orc_trk_word(seed, stream, i, j), W);
        uint64_t run = 0;
        int64_t pick = -1;
        for (int64_t c = 0; c < nc; ++c) {
            run += cs[c].w;
            if (run > r) { pick = c; break; }
        }
        int64_t k = cs[pick].k;
        if (k < 0) break; /* the origin: the walk is complete */
        int32_t x = w.wu[k], tk = w.wt[k];
        int64_t hk = w.head[k];
        if (x != s && x != z && nodeV) nodeV[x]++;
        if (edgeV) edgeV[w.wid[k]]++;
        expect = cs[pick].w;
        if (x == s && opt != OPT_FM) break; /* the origin */
        /* next candidates: the appearances of x counted as tails of k */
        memset(cand_app, 0, (size_t)(w.A ? w.A : 1));
        for (int64_t b = w.app_off[x]; b < w.app_off[x + 1] && w.app_time[b] < tk; ++b)
            if (arc_counted(&w, opt, s, b, hk)) cand_app[b] = 1;
        origin = (x == s) && arc_counted(&w, opt, s, -1, hk);
    }
    if (ret && nodeV) memset(nodeV, 0, sizeof(uint64_t) * (size_t)n);
    if (ret && edgeV) memset(edgeV, 0, sizeof(uint64_t) * (size_t)g->m);
    free(cs);
    free(cand_app);
    pws_free(&w);
    return ret;
}

/* ------------------------------------------------------------------------ */
/* the RTB estimator (appendix on other estimators)                          */

/*
 * One source: nodeF[v] = (1/(n-1)) * sum over targets z != s of f(v|s,z)
 * (orc_pair's N(v)/sigma_sz, unreachable targets adding 0), edgeF[e] (original
 * edge ids) likewise; the sums over targets are double-double.  *reached
 * gets the number of targets s reaches.  Returns 0; 1 if some target's
 * counts saturated (the source is void: rows zero); -1 on bad arguments.
 */
int orc_rtb(const orc_graph *g, int32_t opt, int32_t t0, int32_t t1, int32_t s, int32_t mode, double *nodeF,
            double *edgeF, int64_t *reached, int32_t nthreads) {
    int32_t n = g->n;
    int64_t m = g->m;
    if (s < 0 || s >= n || opt < 0 || opt > 3) return -1;
    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    double *hi = (double *)calloc((size_t)nt * (size_t)(n + m), sizeof(double));
    double *lo = (double *)calloc((size_t)nt * (size_t)(n + m), sizeof(double));
    int64_t nreach = 0, nsat = 0;
#pragma omp parallel num_threads(nt) reduction(+ : nreach, nsat)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *h = hi + (size_t)tid * (size_t)(n + m), *l = lo + (size_t)tid * (size_t)(n + m);
        uint64_t *nN = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
        uint64_t *eN = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m ? m : 1));
#pragma omp for schedule(static)
        for (int32_t z = 0; z < n; ++z) {
            if (z == s) continue;
            orc_record rec;
            orc_pair(g, opt, t0, t1, s, z, mode, &rec, nN, eN);
            if (!rec.reachable) continue;
            nreach++;
            if (rec.flags & REC_OVERFLOW) { nsat++; continue; }
            double sg = (double)rec.sigma;
            for (int32_t v = 0; v < n; ++v)
                if (nN[v]) dd_add(&h[v], &l[v], (double)nN[v] / sg);
            for (int64_t e = 0; e < m; ++e)
                if (eN[e]) dd_add(&h[n + e], &l[n + e], (double)eN[e] / sg);
        }
        free(nN);
        free(eN);
    }
    /* threads' sums in thread order, then the 1/(n-1) */
    for (int64_t x = 0; x < n + m; ++x) {
        double H = 0, L = 0;
        for (int t = 0; t < nt; ++t) {
            dd_add(&H, &L, hi[(size_t)t * (size_t)(n + m) + (size_t)x]);
            dd_add(&H, &L, lo[(size_t)t * (size_t)(n + m) + (size_t)x]);
        }
        double f = (H + L) / (double)(n - 1);
        if (nsat) f = 0.0;
        if (x < n) { if (nodeF) nodeF[x] = f; }
        else if (edgeF) edgeF[x - n] = f;
    }
    free(hi);
    free(lo);
    if (reached) *reached = nreach;
    return nsat ? 1 : 0;
}
