/*
 * mantra.h -- C ABI of the MI355X temporal-betweenness hot path.
 *
 * The library estimates the temporal betweenness centrality of nodes and
 * temporal edges of a directed temporal graph by sampling ordered node pairs
 * (the "ob" estimator of Section 4.1 of the MANTRA paper, arXiv 2304.08356),
 * and stops the sampling with the c-MCERA supremum-deviation bound of
 * Theorem 1 inside the progressive schedule of Algorithm 1.
 *
 * Conventions
 *  - Every call returns a mantra_status (0 = OK, < 0 = error); nothing is
 *    thrown across the ABI.  mantra_last_error() gives a thread-local text.
 *  - Pointers in these signatures are HOST pointers unless stated otherwise.
 *    The library allocates and owns all device memory; the caller owns every
 *    buffer it passes in, and the library copies what it needs before the call
 *    returns (mantra_submit: buffers named in the request must stay valid until
 *    mantra_poll reports the ticket finished).
 *  - Node ids are 0..n-1; a temporal edge is (src, dst, t) with src != dst and
 *    t >= 0.  The edge set is a set (Preliminaries: duplicates are merged).
 *  - Optimalities (Definition 1; fm is an extension, see mantra_opt) are
 *    counted over strict temporal walks: consecutive edges have strictly
 *    increasing times, and the source starts before every edge.
 *  - Path counts are exact integers: uint64, and for the dependency estimator
 *    256-bit words for the pairs whose counts do not fit 64 bits
 *    (MANTRA_REC_WIDE).  A count beyond that is saturated and reported
 *    (MANTRA_REC_OVERFLOW / MANTRA_E_OVERFLOW), never rounded.
 *  - Time windows [t0, t1] are inclusive; the node set and the n(n-1)
 *    normalisation are those of the whole graph.
 */
#ifndef MANTRA_H
#define MANTRA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Temporal path optimality (Definition 1).
 *  SH  : fewest hops.
 *  SFM : earliest arrival first, then fewest hops among those.
 *  PFM : every prefix ending at v_i arrives at the earliest arrival at v_i.
 *  FM  : every walk arriving at the earliest arrival (walks, visits counted
 *        with multiplicity: counting foremost simple paths is #P-hard, see the
 *        Preliminaries).  f(v) may exceed 1, so Theorems 1 and 3 do not cover
 *        it: results carry MANTRA_RES_NO_GUARANTEE. */
typedef enum { MANTRA_SH = 0, MANTRA_FM = 1, MANTRA_SFM = 2, MANTRA_PFM = 3 } mantra_opt;

typedef enum {
    MANTRA_OK = 0,
    MANTRA_PENDING = 1,       /* mantra_poll: not finished yet */
    MANTRA_E_INVALID = -1,    /* bad argument (message says which) */
    MANTRA_E_NODEV = -2,      /* no usable gfx950 device */
    MANTRA_E_OOM = -3,        /* device allocation failed */
    MANTRA_E_OVERFLOW = -4,   /* a sampled pair's count saturated at 2^64-1 */
    MANTRA_E_TOO_LARGE = -5,  /* the request can never fit the memory budget */
    MANTRA_E_INTERNAL = -6,   /* HIP runtime error or broken invariant */
    MANTRA_E_LIMIT = -7       /* a hop count above 65534 */
} mantra_status;

typedef struct mantra_graph mantra_graph; /* opaque, device resident */

/* Per-pair record (bit-exact against the oracle). */
typedef struct {
    int32_t reachable; /* 1 if an optimal walk s -> z exists in the window */
    int32_t t_arr;     /* earliest arrival time among the optimal walks, -1 */
    int32_t hops;      /* fewest hops among the optimal walks, -1 */
    int32_t flags;     /* MANTRA_REC_* */
    uint64_t sigma;    /* number of optimal walks (saturated at 2^64-1) */
} mantra_pair_record;

#define MANTRA_REC_OVERFLOW 1u   /* a count saturated: above 2^256 - 1 for the dependency
                                    estimator (its multiword path), above 2^64 - 1 for the
                                    TRK and RTB estimators */
#define MANTRA_REC_WIDE 16u      /* sigma is above 2^64 - 1 (the record's sigma field then
                                    reads 2^64 - 1): the pair was counted exactly in 256-bit
                                    words (the paper's 128-bit and arbitrary-precision
                                    counts) and its f values are exact quotients */
#define MANTRA_REC_HOPS_LIMIT 4u /* a hop count would exceed 65534 */

/* Build a device-resident temporal graph (Preliminaries: a set of temporal
 * edges (u, v, t) over nodes 0..n-1) from m edges (src[i], dst[i], t[i]),
 * host arrays of int32.  Rejects ids outside [0, n), self-loops and times
 * outside [0, 2^31-2] (MANTRA_E_INVALID); merges exact duplicate triples (the
 * edge set is a set; the count is in mantra_graph_info).  The arrays are
 * copied; the caller keeps them.  *out receives the handle (NULL on error);
 * MANTRA_E_NODEV without a gfx950 device, MANTRA_E_OOM if it does not fit. */
int mantra_graph_create(const int32_t *src, const int32_t *dst, const int32_t *t, int64_t m,
                        int32_t n, uint32_t flags, mantra_graph **out);

/* G independent graphs in one device graph (packed CSR segments).  Graph g
 * has node_count[g] nodes and edges [edge_off[g], edge_off[g+1]) of the
 * arrays, with node ids local to the graph.  Pairs of graph g are sampled
 * among its own nodes; sums are kept per graph. */
int mantra_graph_create_packed(int32_t G, const int32_t *node_count, const int64_t *edge_off,
                               const int32_t *src, const int32_t *dst, const int32_t *t,
                               uint32_t flags, mantra_graph **out);

void mantra_graph_destroy(mantra_graph *g);

/* n, unique edge count, merged duplicates, time span, number of packed graphs */
int mantra_graph_info(const mantra_graph *g, int32_t *n, int64_t *m_unique, int64_t *n_duplicates,
                      int32_t *t_min, int32_t *t_max, int32_t *n_graphs);

/* Test / measurement entry point: the per-pair quantities of Definition 1
 * and of the estimator of Section 4.1 for r explicit pairs (s[q], z[q]) in the
 * window [t0, t1] (host int32 arrays of length r, s[q] != z[q]).  out[r]
 * receives the records.  Optional dense outputs (host, row-major, NULL to
 * skip): node_f[r*n] gets f(v|s,z) = N(v)/sigma and edge_f[r*m] gets
 * f(e|s,z) (Appendix, temporal edges) per input edge index (duplicates share
 * their merged edge's value), for pairs whose counts did not saturate; at
 * most 4e9 doubles each (MANTRA_E_INVALID beyond).  For packed graphs,
 * graph[q] names the pair's graph (NULL for a single graph) and node ids are
 * local to it.  Records of saturated pairs carry MANTRA_REC_OVERFLOW; the
 * call itself still returns MANTRA_OK. */
int mantra_count_pairs(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r,
                       const int32_t *graph, const int32_t *s, const int32_t *z,
                       mantra_pair_record *out, double *node_f, double *edge_f);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture of the surrounding work, tight serving loops, harnesses that
 * forbid hipMalloc): the records of mantra_count_pairs (no dense outputs)
 * computed without any device allocation.  Every buffer beyond the graph --
 * the per-pair node state and arc records of up to 64 workgroups, the launch
 * counters, the pairs and the records -- lives in one device array of the
 * library, 256 MiB, that each GPU holds from the library's load until the
 * process ends.  A workgroup holds an arc record for every edge of the
 * graph, so the graph must fit: one workgroup needs 28 B per node (+1 bit
 * per node above 65,536 nodes) + 32 B per edge of the longest tick + 32 B per
 * edge, and the pairs 36 B each; beyond the array MANTRA_E_TOO_LARGE.  Pairs
 * whose counts pass 2^64 carry MANTRA_REC_OVERFLOW (no 256-bit re-count: that
 * path allocates).  Calls on one GPU share the array and would race; the
 * library serializes them per device.  Arguments, outputs and the other
 * errors as mantra_count_pairs; blocking. */
int mantra_count_pairs_static(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r,
                              const int32_t *graph, const int32_t *s, const int32_t *z,
                              mantra_pair_record *out);

/* The TRK estimator's walks for r explicit pairs (arguments and outputs as
 * mantra_count_pairs): one optimal walk per reachable pair, drawn backwards
 * from z with probability 1/sigma_sz (the appendix's path sampler, Theorem on
 * the path sampler).  Step j of pair q draws w = the SplitMix64 output
 * (q * 2^16 + j + 1) of the generator started at the (2^20 + 1)-th output of
 * the one started at seed, takes r = floor(w * W / 2^64) for the step's total
 * weight W, and picks the first candidate arc, in the order (time, input
 * head id, input tail id), whose running weight exceeds r.  node_f[q*n + v]
 * gets the walk's internal visits of v, edge_f[q*m + e] its uses of e. */
int mantra_sample_paths(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r,
                        const int32_t *graph, const int32_t *s, const int32_t *z, uint64_t seed,
                        mantra_pair_record *out, double *node_f, double *edge_f);

/* The RTB estimator's f for r explicit sources s[q] (node ids local to
 * graph[q], or graph 0 when graph is NULL): node_f[q*n + v] =
 * (1/(n-1)) sum_{z != s} sigma_sz(v)/sigma_sz and edge_f[q*m + e] likewise,
 * computed in double precision from one forward sweep of s to the end of
 * [t0, t1] and one reverse sweep over all targets.  out[q]: reachable = 1 if
 * s reaches any node, sigma = the number of nodes it reaches, t_arr = hops =
 * -1; MANTRA_REC_OVERFLOW if a count on the way saturated (f rows are then
 * zero). */
int mantra_source_dependencies(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r,
                               const int32_t *graph, const int32_t *s, mantra_pair_record *out,
                               double *node_f, double *edge_f);

/* One estimation request. */
typedef struct {
    mantra_opt opt;
    int32_t t0, t1;        /* inclusive window; t1 < t0 means the whole span */
    double eps, delta;     /* accuracy and failure probability, in (0, 1) */
    uint64_t seed;         /* pairs and Rademacher signs are functions of it */
    int32_t c;             /* Monte Carlo trials of the c-MCERA, 1..64 (0: 25) */
    int64_t s1;            /* first sample size override (0: from the bound) */
    int64_t max_samples;   /* cap on the sample size (0: none) */
    int64_t fixed_r;       /* > 0: exactly this many pairs, no progressive loop */
    uint32_t flags;        /* MANTRA_F_* */
    double *node_bc;       /* out [n] (packed: [sum of n_g]), caller owned */
    double *edge_bc;       /* out [m] input edge order, or NULL */
} mantra_request;

#define MANTRA_F_EDGE_BC 1u /* also estimate temporal-edge betweenness */
#define MANTRA_F_TRK 2u     /* the TRK estimator (appendix on other estimators):
                               per sampled pair one optimal walk, drawn with
                               probability 1/sigma_sz, and f(v) = its internal
                               visits of v, f(e) = its uses of e, instead of
                               the ob estimator's N(v)/sigma_sz.  Unbiased for
                               the same betweenness; f in {0, 1} except for fm
                               walks, which may revisit a node */
#define MANTRA_F_RTB 4u     /* the RTB estimator (appendix on other estimators):
                               each sample is a source s (uniform over the
                               nodes), swept to the window's end, with
                               f(v) = (1/(n-1)) sum over targets z != s of
                               sigma_sz(v)/sigma_sz and f(e) likewise; the
                               sample sizes count sources */

typedef struct {
    double *node_bc;       /* estimates of every node (host, [n], input node order;
                              packed graphs: [sum of n_g]).  mantra_estimate: set by
                              the caller, required; mantra_run and mantra_poll: the
                              request's buffer, now filled */
    double *edge_bc;       /* estimates of every temporal edge (host, [m], input edge
                              order), or NULL.  mantra_estimate: set by the caller,
                              optional (NULL: no temporal-edge estimates); mantra_run
                              and mantra_poll: the request's buffer, now filled */
    int32_t status;        /* mantra_status of the request */
    uint32_t flags;        /* MANTRA_RES_* */
    int64_t samples;       /* |S| at the stop */
    int64_t rounds;        /* progressive rounds run */
    int64_t omega;         /* Theorem 3 sample size bound */
    int64_t s_boot;        /* bootstrap pairs s' */
    int64_t s1;            /* first sample size */
    int64_t n_overflow;    /* sampled pairs whose counts saturated */
    int64_t n_reachable;   /* sampled pairs with sigma > 0 */
    int64_t window_edges;  /* temporal edges swept, summed over pairs */
    int64_t arcs;          /* appearance-DAG arcs recorded, summed over pairs */
    double xi;             /* supremum-deviation bound at the stop */
    double rho_hat, v_hat; /* bootstrap estimates */
    double wimpy, mcera;   /* last round's W and R^c */
    double gpu_ms;         /* device time of the sweep kernels */
    double latency_ms;     /* submit -> finish (serving) or call duration */
} mantra_result;

#define MANTRA_RES_NO_GUARANTEE 1u /* fm: Theorems 1 and 3 do not apply */
#define MANTRA_RES_STOP_XI 2u      /* stopped because xi <= eps */
#define MANTRA_RES_STOP_OMEGA 4u   /* stopped because |S| >= omega */

/* Algorithm 1 (bootstrap, sample-size bound of Theorem 3, progressive
 * rounds stopped by the c-MCERA bound of Theorem 1) on the whole time span
 * with the experimental defaults (c = 25), blocking: the problem statement of
 * Section 3 (input the graph, the optimality, eps, delta; output the
 * estimates of every node).  The caller sets out->node_bc (host, [n],
 * caller-owned; NULL is MANTRA_E_INVALID) and out->edge_bc (host, [m], or
 * NULL: no temporal-edge estimates); the call fills them and the rest of
 * *out.  MANTRA_E_OVERFLOW (estimates NaN) if a sampled pair's count
 * saturated. */
int mantra_estimate(mantra_graph *g, mantra_opt opt, double eps, double delta, uint64_t seed,
                    mantra_result *out);

/* Blocking run of one request: Algorithm 1 as above, or with fixed_r > 0 a
 * fixed sample of fixed_r pairs (per packed graph), over the request's window,
 * with c sign vectors and, with MANTRA_F_EDGE_BC, temporal-edge estimates in
 * edge_bc[m] (input edge order).  Same errors as mantra_estimate.  A request
 * whose sample holds a saturated pair stops at the end of that phase (the
 * bootstrap or a round) with MANTRA_E_OVERFLOW: its estimates are void, so
 * it runs no further rounds (served requests alike). */
int mantra_run(mantra_graph *g, const mantra_request *req, mantra_result *out);

/* Result of mantra_distances (appendix on temporal distance metrics,
 * Algorithm 2).  d(u, v) is the number of temporal edges of the
 * (*)-optimal walks from u to v (for sfm: the fewest among the walks
 * arriving first; for fm: the fewest among all walks arriving first; for pfm:
 * that of the prefix-foremost walks).  With R[h] = (n / r) * (sampled pairs
 * (u, v), v != u, with d(u, v) <= h), the paper's R array: */
typedef struct {
    int64_t sources;        /* r */
    int64_t reached_pairs;  /* sampled (source, node) pairs joined by a walk */
    int32_t d_lb;           /* D_LB: the largest distance seen (a lower bound on
                               the (*)-temporal diameter D; VD = D + 1) */
    int32_t d_tau;          /* D_tau: least h with R[h] / R[D_LB] >= tau; -1 if
                               no sampled pair is reachable */
    double zeta;            /* connectivity rate R[D_LB] / (n (n - 1)) */
    double psi;             /* average distance over reachable pairs,
                               sum_h h (R[h] - R[h-1]) / R[D_LB]; 0 if none */
    double rho;             /* average internal nodes over all n (n - 1)
                               ordered pairs, sum_h (h - 1)(R[h] - R[h-1])
                               / (n (n - 1)) (unreachable pairs count 0) */
    int64_t window_edges;   /* temporal edges swept, summed over sources */
    double gpu_ms;          /* device time of the sweep */
} mantra_distance_result;

/* Algorithm 2: r sources drawn uniformly (with replacement) from the seed's
 * source stream, each swept forward from its first departure to the end of
 * [t0, t1] (t1 < t0: the whole span) without a target; the distances of every
 * node it reaches form the per-hop counts, from which the quantities above
 * follow.  hist (host, may be NULL when hist_len = 0) receives the raw counts:
 * hist[h] = sampled pairs at distance exactly h for h < hist_len - 1, the
 * last entry every larger distance.  tau in [0, 1].  Single graphs only
 * (packed: MANTRA_E_INVALID), n >= 2, 1 <= r <= 2^31 - 1.  MANTRA_E_LIMIT if
 * a distance exceeds 65534.  Blocking. */
int mantra_distances(mantra_graph *g, mantra_opt opt, int32_t t0, int32_t t1, int64_t r, uint64_t seed,
                     double tau, uint64_t *hist, int32_t hist_len, mantra_distance_result *out);

/* Serving (not in the paper: a request loop around Algorithm 1).  Non-blocking
 * submission to the graph's scheduler thread, which batches the phases of all
 * admitted requests into shared sweep launches.  Admission is FIFO by the
 * device memory a request's sums need (8n(2+c) + 8m with edge estimates,
 * + 24n for the bootstrap); a request that can never fit the budget returns
 * MANTRA_E_TOO_LARGE at once, invalid requests MANTRA_E_INVALID.  The
 * buffers named in the request must stay valid until the ticket finishes.
 * mantra_poll waits up to timeout_ms (0: no wait, < 0: forever) and returns
 * MANTRA_OK (result filled, ticket consumed), MANTRA_PENDING, or the request's
 * error (result filled, ticket consumed); MANTRA_E_INVALID for an unknown or
 * consumed ticket.  Destroying the graph fails the requests it still holds
 * (MANTRA_E_INTERNAL). */
int mantra_submit(mantra_graph *g, const mantra_request *req, uint64_t *ticket);
int mantra_poll(uint64_t ticket, mantra_result *out, int32_t timeout_ms);

/* Serving configuration: device bytes the scheduler may use for per-request
 * sums (0: the default, three quarters of the memory left free once the slab
 * pool -- the per-pair node state and arc buffers that every launch shares,
 * 75% of the device -- is reserved), maximum concurrent requests. */
int mantra_serve_config(mantra_graph *g, uint64_t mem_budget_bytes, int32_t max_active);

/* Launch configuration of the sweep (it changes how the work is scheduled,
 * never a result). */
typedef struct {
    int32_t n_slabs;      /* persistent workgroups per launch, each one pair at a
                             time (0: as many as fit the device) */
    int64_t arc_cap;      /* appearance-DAG arc records of each workgroup's own
                             buffer (0: 2^18, or up to 2^20 where the grid the
                             device keeps resident still fits half of the slab
                             budget with it; at most one per edge of the graph);
                             a pair with more takes chunks of 2^18 arcs from a
                             pool the launch shares (the rest of the slab
                             budget).  A pair that finds none free is re-run
                             after the launch, alone with the other such pairs
                             on the same pool, and if it again finds none, with
                             room for every edge */
    int32_t order;        /* MANTRA_ORDER_*: the order pairs are handed out in */
    int32_t graph_rounds; /* 1: the progressive rounds of a blocking request
                             replay one captured HIP graph (counters, order,
                             sweep and reduction) */
    int32_t per_pair_launch; /* 1: the unbatched form, one single-workgroup
                                launch per pair (a baseline for measurement) */
    int32_t hub_nodes;    /* forward state of the hub_nodes highest-degree nodes
                             of each pair kept in LDS (0: none, at most 4,096) */
    int32_t wide_counts;  /* pairs whose 64-bit counts saturate, counted again in
                             256-bit words (dependency estimator): MANTRA_WIDE_* */
    int32_t no_arc_chunks; /* 1: no shared arc chunks (every pair beyond its
                              workgroup's own buffer is re-run) */
    int64_t arc_chunks;   /* > 0: at most this many shared arc chunks (0: the
                             rest of the slab budget) */
} mantra_launch_config;

#define MANTRA_WIDE_NONE 0    /* reported as saturated */
#define MANTRA_WIDE_NOT_FM 1  /* sh, sfm and pfm pairs (default): fm walk counts grow
                                 exponentially with the ticks and mostly pass 2^256 too */
#define MANTRA_WIDE_ALL 2     /* every optimality */

#define MANTRA_ORDER_LONGEST_FIRST 0 /* decreasing estimated window (default) */
#define MANTRA_ORDER_DRAWN 1         /* sample order */

int mantra_set_launch(mantra_graph *g, const mantra_launch_config *cfg);
/* the configuration in force, automatic values resolved */
int mantra_get_launch(const mantra_graph *g, mantra_launch_config *cfg);

/* Autotuner: times the sweep on a calibration sample of sample_pairs pairs
 * (0: four times the largest candidate grid, two times where device memory
 * bounds the grid) drawn for optimality opt from the bootstrap stream of
 * seed, under candidate grid sizes (1, 7/8, 3/4, 5/8 and 1/2 of the
 * automatic grid; where device memory, not residency, bounds that grid, also
 * 3/2 and 2 times it, up to the resident workgroups, with smaller arc
 * buffers) and both pair orders.  Where memory bounds the grid, candidates
 * are compared by the grid's mean busy time (a steady-state rate; the order
 * is then longest first) rather than by the sample's time, which its longest
 * pairs decide.  Then hub nodes in LDS: where residency bounds the grid, 256
 * of them at the best of those grids, and 256, 512 and 1,024 each at the
 * grid resident with that LDS (all and 7/8 of it); where memory bounds it,
 * 1,024, 2,048 and 4,096 at the best grid (or the grid still resident).  Keeps the fastest as the graph's launch
 * configuration and writes it to *best (may be NULL).  Blocking, for about a
 * dozen runs of the sample (minutes on graphs of millions of nodes, where a
 * smaller sample_pairs shortens it); results of later calls do not depend on
 * the choice. */
int mantra_autotune(mantra_graph *g, mantra_opt opt, int64_t sample_pairs, uint64_t seed,
                    mantra_launch_config *best);

/* Work and timing of the last blocking call on g: device time of the sweep
 * kernel launches (HIP events on the graph's stream), their count, the
 * totals over its pairs of swept window edges, recorded appearance-DAG arcs,
 * touched nodes (N(v) > 0) and touched temporal edges (N(e) > 0), the load
 * balance of the persistent grid (busy time of its workgroups over
 * workgroups x launch span, averaged over launch time), the forward
 * sweep's batches of up to 64 window edges that loaded node state and that
 * were skipped (no reached tail), and the forward sweeps' share of the
 * workgroups' time in pairs (the rest: reverse sweeps, walks and the
 * accumulation).  Any pointer may be NULL. */
int mantra_last_timing(const mantra_graph *g, double *sweep_ms, int64_t *launches,
                       int64_t *window_edges, int64_t *arcs, int64_t *touched_nodes,
                       int64_t *touched_edges, double *balance, int64_t *live_batches,
                       int64_t *skipped_batches, double *forward_share);

/* Test entry point: sets the pair serial of every workgroup of the graph's
 * slab pool (allocating the pool first), as a pool in use for billions of
 * pairs would hold it.  Slab state words are tagged with this 32-bit
 * counter; the library clears the pool's tagged state before it could wrap,
 * so results never depend on it. */
int mantra_debug_stamps(mantra_graph *g, uint32_t serial);

const char *mantra_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MANTRA_H */
