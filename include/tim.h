/*
 * tim.h — C ABI of the MI355X (gfx950) TIM / TIM+ engine.
 *
 * Paper: Tang, Xiao, Shi, "Influence Maximization: Near-Optimal Time
 * Complexity Meets Practical Efficiency", SIGMOD 2014.
 *
 * The library computes, on one GPU, the data-parallel hot path of TIM/TIM+:
 * random reverse-reachable (RR) sets (Definitions 1-2), their widths and
 * kappa values (Equation (1), Equation (8)), KptEstimation (Algorithm 2),
 * RefineKPT (Algorithm 3) and greedy maximum-coverage NodeSelection
 * (Algorithm 1), assembled into TIM (Section 3.3) and TIM+ (Section 4.1).
 *
 * Results are deterministic functions of (graph, model, k, eps, ell, seed):
 * every random number is a Philox4x32-10 block keyed by the seed and
 * addressed by (phase, kind, index, set id), so a set can be regenerated
 * anywhere and the output does not depend on launch geometry or timing.
 *   key     = (seed & 0xFFFFFFFF, seed >> 32)
 *   counter = (idx & 0xFFFFFFFF, phase<<24 | kind<<16 | (idx>>32 & 0xFFFF),
 *              set & 0xFFFFFFFF, set >> 32)
 *   kind 0: root of the set (idx 0); root = floor(X64 * n / 2^64) with
 *           X64 = word1<<32 | word0
 *   kind 1: IC coins, idx = e >> 2 for in-CSR edge e; word e & 3 decides e:
 *           live iff word <= t(e) (t(e) = uint32 threshold; weighted cascade:
 *           t = floor(2^32 / indeg(dst)) - 1)
 *   kind 2: LT pick at node v (idx = v); in-edge off[v] + floor(X64*indeg/2^64)
 *   kind 3: triggering-set pick at node v (idx = v), by word 0 (general
 *           triggering model; see tim_graph_set_triggering)
 *   phase i in [1, 62]: KptEstimation round i; 63: RefineKPT's fresh sets;
 *   64: NodeSelection's sets.  Set ids start at 0 in every phase.
 *
 * Conventions for every call:
 *   - Status codes only; nothing is thrown across the ABI.  On failure,
 *     tim_last_error() returns a message for the calling thread.
 *   - "host" pointers are ordinary CPU memory owned by the caller and only
 *     read or written during the call.  "device" pointers are GPU memory
 *     owned by the caller (for example torch tensors on the ROCm device).
 *   - All GPU work is ordered on the context's stream; every call returns
 *     after that work has finished (results are final on return).
 *   - One context per host thread; calls on one context must not overlap.
 *   - Node ids are int32 (n < 2^31), CSR offsets int64 (m < 2^32).
 */
#ifndef TIM_H_
#define TIM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TIM_ABI_VERSION 1

typedef enum {
  TIM_OK = 0,
  TIM_EINVAL = 1,    /* an argument is out of range or a graph is malformed */
  TIM_ENOMEM = 2,    /* a host or device allocation failed */
  TIM_EBUDGET = 3,   /* the work does not fit the context's device-memory budget */
  TIM_EDEVICE = 4,   /* a HIP runtime call or kernel launch failed */
  TIM_ECAPACITY = 5  /* a caller-provided output buffer is too small */
} tim_status;

typedef enum {
  TIM_MODEL_IC = 0,     /* independent cascade (Section 2.1) */
  TIM_MODEL_LT = 1,     /* linear threshold: a triggering model whose triggering set
                           is one in-neighbour or none (Section 4.2; Section 7.1);
                           in-weights 1/indeg(v) unless tim_graph_set_lt_weights
                           gave the graph others */
  TIM_MODEL_TRIGGER = 2 /* general triggering model (Section 4.2): each node draws its
                           triggering set from the explicit distribution that
                           tim_graph_set_triggering gave the graph (tim_run and the
                           phase, sampling and spread calls; not batches or servers) */
} tim_model;

enum { TIM_PHASE_REFINE = 63, TIM_PHASE_SELECT = 64 };

enum {
  TIM_FLAG_PLAIN = 1u,      /* TIM (Section 3.3): skip RefineKPT, theta = lambda/KPT* */
  TIM_FLAG_ELL_ADJUST = 2u  /* scale ell by 1 + ln2/ln n (TIM) or 1 + ln3/ln n (TIM+)
                               so that the overall success probability is 1 - n^-ell
                               (Sections 3.3 and 4.1) */
};

#define TIM_MAX_ROUNDS 64

typedef struct tim_ctx tim_ctx;
typedef struct tim_graph tim_graph;

/* Per-launch totals of a batch of RR sets. */
typedef struct {
  uint64_t count;        /* sets generated */
  uint64_t kappa_sum_lo; /* sum over sets of kappa(R) * 2^53, low 64 bits (exact) */
  uint64_t kappa_sum_hi; /* ... high 64 bits */
  uint64_t width_sum;    /* sum of w(R) = edges examined (Equation (1)) */
  uint64_t node_sum;     /* sum of |R| */
  uint64_t covered;      /* sets that meet the seed set (coverage mode only) */
  uint64_t deferred;     /* sets finished by the large-set pass */
} tim_batch_stats;

/* KptEstimation (Algorithm 2). */
typedef struct {
  int32_t i_max;   /* number of rounds allowed: floor(log2 n) - 1 */
  int32_t i_last;  /* round that stopped (i_max if none did) */
  uint64_t c_last; /* c_i of that round */
  double kpt_star; /* KPT*; 1.0 if no round stopped */
  uint64_t round_c[TIM_MAX_ROUNDS];      /* indexed by round i (entry 0 unused) */
  uint64_t round_sum_lo[TIM_MAX_ROUNDS]; /* exact sum of kappa * 2^53, low/high words */
  uint64_t round_sum_hi[TIM_MAX_ROUNDS];
  uint64_t round_width[TIM_MAX_ROUNDS];
  uint64_t round_nodes[TIM_MAX_ROUNDS];
} tim_kpt_result;

/* RefineKPT (Algorithm 3). */
typedef struct {
  double eps_prime;       /* 5 * cbrt(ell * eps^2 / (k + ell)) */
  double lambda_prime;    /* (2 + eps') * ell * n * ln n / eps'^2 */
  uint64_t theta_prime;   /* ceil(lambda' / KPT*) */
  uint64_t covered_prime; /* fresh sets that meet S'_k */
  double kpt_prime;       /* (covered'/theta') * n / (1 + eps') */
  double kpt_plus;        /* max(KPT', KPT*) */
} tim_refine_result;

/* NodeSelection (Algorithm 1).  The collection is kept in device memory
 * with its inverted index when it fits the context's budget (without one:
 * the free device memory).  Otherwise sets [0, resident_sets) are kept and
 * the rest is regenerated from its keys in chunks of chunk_sets sets, once
 * for the initial counts and once after every greedy step but the last
 * (regenerated_sets counts the generations beyond the first).  Sets are a
 * function of (seed, phase, id), so the seeds and gains do not depend on
 * this. */
typedef struct {
  uint64_t theta;     /* sets generated */
  uint64_t nodes;     /* total size of the RR collection */
  uint64_t width;     /* total width (edges examined) */
  uint64_t covered;   /* sets covered by the k seeds = sum of gains */
  uint64_t store_bytes; /* device bytes held for the collection and its index */
  uint64_t resident_sets;    /* sets kept with their inverted index (theta if all) */
  uint64_t chunk_sets;       /* sets per regenerated chunk (0 if none) */
  uint64_t regenerated_sets; /* set generations beyond the first */
} tim_select_result;

/* Everything tim_run computes, with per-phase GPU times in milliseconds. */
typedef struct {
  double ell_used;
  double lambda;
  tim_kpt_result kpt;
  tim_refine_result refine;
  tim_select_result select;
  int32_t s_prime[128]; /* S'_k of RefineKPT (first min(k,128) entries) */
  double ms_kpt, ms_refine, ms_select_sample, ms_select_index, ms_select_greedy, ms_total;
  uint64_t sets_total;  /* RR sets generated over all phases */
  uint64_t width_total; /* edges examined over all phases */
} tim_report;

/* ---- context ------------------------------------------------------------ */

/* Creates a context on HIP device `device`.  `stream` is a hipStream_t to
 * order work on (NULL: the library creates its own).  `hbm_budget_bytes`
 * caps the device memory the library allocates for RR sets, their index and
 * the sampler's work space (0: no cap; the free device memory then bounds
 * the RR collection).  The graph is not counted.  A collection that does
 * not fit is processed in regenerated chunks (see tim_select_result);
 * TIM_EBUDGET means the budget is too small even for that.  Returns
 * TIM_EDEVICE if the device cannot be used. */
tim_status tim_ctx_create(int device, void *stream, uint64_t hbm_budget_bytes, tim_ctx **out);
void tim_ctx_destroy(tim_ctx *ctx);

/* Message of the last failing call on this thread ("" if none). */
const char *tim_last_error(void);

/* Bytes of device memory currently held by the context (graphs excluded). */
uint64_t tim_ctx_device_bytes(const tim_ctx *ctx);

/* Most RR sets a greedy (RefineKPT's and NodeSelection's) keeps resident
 * with their inverted index; the rest is regenerated in chunks between
 * greedy steps, as when the collection exceeds the budget.  UINT64_MAX (the
 * default) sets no limit; 0 regenerates every set.  Results do not depend on
 * it. */
tim_status tim_set_resident_limit(tim_ctx *ctx, uint64_t max_sets);

/* ---- tuning -------------------------------------------------------------- */

/* What tim_autotune measured and chose. */
typedef struct {
  int32_t seg_lanes;   /* lanes per IC set in the first sampler tier: 4, 8, 16, 32 or 64 (with it come
                          the sizes a set may reach before a later tier takes it: a 64/128/128/256/512-
                          node queue and 256/512/512/1024/2048 four-edge groups) */
  uint32_t slice_cap;  /* largest node-pool slice a wavefront reserves when storing sets */
  double ms_width[5];  /* IC: one width-mode launch of `sets` sets with 4, 8, 16, 32, 64 lanes (0 for LT) */
  double ms_emit[4];   /* one stored-set launch with slice caps 512, 1024, 2048, 4096 */
  double ms_lanes_emit[5]; /* IC: one stored-set launch of `sets` sets with 4, 8, 16, 32, 64 lanes (0 for LT) */
} tim_tune_result;

/* Times the context's sampler shapes on graph g and keeps the fastest for
 * the context's later calls: first the IC first-tier lanes per set (the
 * wave-per-set thresholds), by the sum of one width-mode launch (as the
 * KptEstimation rounds run) and one stored-set launch (as the last round
 * kept for RefineKPT and NodeSelection run), then the node-pool slice size
 * (stored sets).  Each candidate runs `sets` sets (phase 66, a fixed
 * seed; the sets are dropped) once untimed and three times timed; the best
 * wall time wins if it beats the current shape by 3% or more (else the
 * current one stays).  Results of every call do not depend on these shapes.
 * Requires 4096 <= sets <= 2^26.  out (host) may be NULL. */
tim_status tim_autotune(tim_ctx *ctx, const tim_graph *g, int model, uint64_t sets, tim_tune_result *out);

/* ---- profile ------------------------------------------------------------ */

/* Work and GPU time of one sampler kernel (one model, one mode), summed over
 * its launches since profiling was enabled.  Times come from HIP events
 * recorded on the context's stream around each launch.  "bytes" are the
 * algorithmic bytes of the sets the kernel finished itself (sets deferred to
 * the large-set pass are excluded).  IC: per node 16 (its two CSR offsets),
 * per examined in-edge 4 (its source; +4 for its threshold when the graph
 * carries per-edge thresholds).  LT: per node 16 + 4 (offsets and the one
 * picked source).  Both: when sets are stored, 4 per node plus 12 per set. */
typedef struct {
  uint64_t launches;
  double kernel_ms;
  uint64_t sets, nodes, edges, bytes;
  uint64_t large_launches; /* large-set pass launches and time */
  double large_ms;
  uint64_t deferred;       /* sets it finished */
} tim_kernel_profile;

typedef struct {
  tim_kernel_profile sampler[2][3]; /* [model][0: widths, 1: stored sets, 2: coverage] */
  uint64_t index_calls;             /* inverted-index builds + greedy runs */
  double index_ms, greedy_ms;
  tim_kernel_profile ic_wide[3];    /* IC launches of fewer than 262144 sets (widths, coverage), which run
                                       the 64-lane first tier; sampler[0][] holds the others */
  tim_kernel_profile grouped[2];    /* [model] multi-job launches that run several early KptEstimation rounds
                                       at once, one job per round; sets counts every set they sampled,
                                       those of rounds past the stopping one included */
} tim_profile;

/* Turns per-launch timing on (on != 0) or off, and clears the counters. */
tim_status tim_profile_enable(tim_ctx *ctx, int on);
/* Copies the counters (host out). */
tim_status tim_profile_read(const tim_ctx *ctx, tim_profile *out);

/* ---- graph (Table 1: G^T as in-edge CSR) --------------------------------- */

/* Copies a directed graph to the device.
 *   in_off  host int64[n+1]: in-edges of v are positions in_off[v]..in_off[v+1]-1
 *   in_src  host int32[m]:   source of each in-edge, sorted by (dst, src),
 *                            no self-loops, no repeated edges
 *   ic_thr  host uint32[m] or NULL: IC threshold t(e) = floor(p(e)*2^32) - 1 of
 *           each edge (p(e) = (t+1)/2^32).  NULL selects the weighted cascade
 *           p(e) = 1/indeg(dst) of Section 7.1.  LT ignores it.
 * Requires 2 <= n < 2^31 and 1 <= m <= 2^32 - 16 (edge positions are 32-bit
 * inside the kernels).  TIM_EINVAL names the first violation. */
tim_status tim_graph_upload(tim_ctx *ctx, int64_t n, int64_t m, const int64_t *in_off, const int32_t *in_src,
                            const uint32_t *ic_thr, tim_graph **out);
void tim_graph_free(tim_graph *g);

/* LT with in-weights (Section 7.1: a random weight per in-edge, normalized
 * so that each node's weights sum to 1; weights summing below 1 leave the
 * empty triggering set the rest).  lt_thr host uint32[m]: cumulative
 * thresholds over each node's in-edges in CSR order, t_j = floor(C_j * 2^32)
 * - 1 for the cumulative weight C_j, non-decreasing within a node (2^32 - 1
 * at a node's last edge when its weights sum to 1).  The walk at v takes the
 * first in-edge j with x <= t_j, x = word 0 of v's pick draw (kind 2), and
 * stops at v if x > t_{d-1}.  in_off is the graph's host offsets (to check
 * the order).  Later LT calls on g use these weights; NULL restores 1/indeg.
 * TIM_EINVAL names the first decreasing pair. */
tim_status tim_graph_set_lt_weights(tim_ctx *ctx, tim_graph *g, const uint32_t *lt_thr, const int64_t *in_off);

/* General triggering model (Section 4.2: node v is activated when a node of
 * its triggering set T(v), a random subset of its in-neighbours, is active).
 * The distribution of T(v) is given explicitly per node, all arrays host:
 *   toff int64[n+1]: the outcomes of v are j in [toff[v], toff[v+1])
 *   tthr uint32[J]:  cumulative thresholds, non-decreasing within a node:
 *                    t_j = floor(C_j * 2^32) - 1 for the cumulative
 *                    probability C_j of v's outcomes up to j
 *   tset int64[J+1]: outcome j's members are tmem[tset[j] .. tset[j+1])
 *   tmem uint32[...]: local in-edge indices i (the in-edge in_off[v] + i),
 *                    strictly increasing within an outcome
 *   in_off:          the graph's host offsets (to check the members)
 * With x = word 0 of v's draw of kind 3, T(v) is the first outcome with
 * x <= t_j, and empty if there is none (probability 1 - C of v's last
 * outcome), so outcome j has probability (t_j - t_{j-1}) / 2^32.  An RR set
 * is the randomized BFS of Section 4.2: every dequeued node draws T(v) and
 * its unvisited members join.  Widths stay sum of in-degrees (Equation (1)).
 * toff NULL removes the distribution.  TIM_EINVAL names the first violation
 * (J < 2^32); nothing changes then. */
tim_status tim_graph_set_triggering(tim_ctx *ctx, tim_graph *g, const int64_t *toff, const uint32_t *tthr,
                                    const int64_t *tset, const uint32_t *tmem, const int64_t *in_off);

/* ---- RR sets (Definitions 1-2; Section 3.1; Section 4.2) ---------------- */

/* Generates sets [first, first+count) of (seed, phase) and writes them as a
 * CSR in caller device memory:
 *   d_set_off  device int64[count+1]: set j is d_nodes[d_set_off[j] .. d_set_off[j+1])
 *   d_nodes    device int32[nodes_capacity]: the nodes of each set (order
 *              within a set unspecified)
 *   d_widths   device uint64[count] or NULL: w(R) of each set (Equation (1))
 * *total_nodes (host) receives the total size.  If it exceeds nodes_capacity,
 * nothing is written to d_nodes and TIM_ECAPACITY is returned; call again with
 * a buffer of *total_nodes entries.  stats (host, nullable) receives totals. */
tim_status tim_sample_rr(tim_ctx *ctx, const tim_graph *g, int model, uint64_t seed, uint32_t phase, uint64_t first,
                         uint64_t count, int64_t *d_set_off, int32_t *d_nodes, uint64_t nodes_capacity,
                         uint64_t *d_widths, uint64_t *total_nodes, tim_batch_stats *stats);

/* Generates sets [first, first+count) of (seed, phase) without storing them,
 * and accumulates kappa(R) = 1 - (1 - w(R)/m)^k (Equation (8)) as the exact
 * integer sum of kappa * 2^53 (kappa in binary64: q = 1 - w/m, q^k by binary
 * exponentiation, no fused multiply-add).  d_widths / d_sizes (device
 * uint64[count] / uint32[count], nullable) receive w(R) and |R| per set. */
tim_status tim_sample_widths(tim_ctx *ctx, const tim_graph *g, int model, uint64_t seed, uint32_t phase,
                             uint64_t first, uint64_t count, int k, uint64_t *d_widths, uint32_t *d_sizes,
                             tim_batch_stats *stats);

/* Generates sets [first, first+count) of (seed, phase) and counts those that
 * contain at least one of the nodes seeds[0..nseeds) (host int32), as in
 * Algorithm 3's test of fresh sets against S'_k.  The count is in stats->covered. */
tim_status tim_sample_cover(tim_ctx *ctx, const tim_graph *g, int model, uint64_t seed, uint32_t phase,
                            uint64_t first, uint64_t count, const int32_t *seeds, int nseeds,
                            tim_batch_stats *stats);

/* ---- greedy maximum coverage (Algorithm 1) ------------------------------ */

/* Runs the greedy on a caller-supplied collection of nsets sets over nodes
 * [0, n) (d_set_off device int64[nsets+1], d_nodes device int32; sets must not
 * repeat a node).  Each step takes the unselected node that covers the most
 * remaining sets (ties: lowest id) and removes the sets it covers; seeds and
 * gains (host int32[k] / uint64[k]) receive the nodes in selection order and
 * the number of sets each one newly covered. */
tim_status tim_max_coverage(tim_ctx *ctx, int64_t n, uint64_t nsets, const int64_t *d_set_off, const int32_t *d_nodes,
                            int k, int32_t *seeds, uint64_t *gains);

/* tim_max_coverage for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same greedy, results identical to tim_max_coverage, with its work
 * arrays (counts, index, marks) in one fixed device array that the library
 * holds on each GPU until the process ends (about 53 MB, located when a
 * context is first created on the device).  It calls no allocator.  Limits
 * of that array: n <= 2^20 nodes, nsets <= 2^22 sets, at most 2^23 entries in
 * all, k <= 1024; larger inputs return TIM_EINVAL and change nothing.  Every
 * call on a GPU uses that GPU's one array (each call clears what it needs),
 * so calls that overlap on one GPU, from any contexts or threads, race and
 * must be serialized by the caller. */
tim_status tim_max_coverage_noalloc(tim_ctx *ctx, int64_t n, uint64_t nsets, const int64_t *d_set_off,
                                    const int32_t *d_nodes, int k, int32_t *seeds, uint64_t *gains);

/* ---- the three phases ---------------------------------------------------- */

/* KptEstimation (Algorithm 2): rounds i = 1 .. floor(log2 n)-1 of
 * c_i = ceil((6*ell*ln n + 6*ln(log2 n)) * 2^i) sets (Equation (9)); stops at
 * the first round whose exact kappa sum S satisfies S * 2^i > c_i * 2^53 and
 * returns KPT* = (S * 2^-53) * n / (2 * c_i); KPT* = 1 if no round stops.
 * Requires 1 <= k <= n, ell >= 0.5. */
tim_status tim_kpt_estimate(tim_ctx *ctx, const tim_graph *g, int model, uint64_t seed, int k, double ell,
                            tim_kpt_result *out);

/* RefineKPT (Algorithm 3): greedy on the sets of round i_last (regenerated
 * from their keys) gives S'_k (s_prime, host int32[k]); theta' fresh sets of
 * phase 63 estimate KPT' and KPT+ = max(KPT', KPT*).  Requires 0 < eps <= 1
 * (the range the paper gives for its eps' rule). */
tim_status tim_refine_kpt(tim_ctx *ctx, const tim_graph *g, int model, uint64_t seed, int k, double eps, double ell,
                          double kpt_star, int i_last, uint64_t c_last, int32_t *s_prime, tim_refine_result *out);

/* NodeSelection (Algorithm 1): theta sets of phase 64, then k greedy steps.
 * seeds / gains: host int32[k] / uint64[k].  out (host) may be NULL. */
tim_status tim_node_select(tim_ctx *ctx, const tim_graph *g, int model, uint64_t seed, int k, uint64_t theta,
                           int32_t *seeds, uint64_t *gains, tim_select_result *out);

/* TIM+ (default) or TIM (TIM_FLAG_PLAIN): KptEstimation, [RefineKPT],
 * theta = ceil(lambda / KPT+ (or KPT*)) with lambda of Equation (4), then
 * NodeSelection.  Requires 1 <= k <= n, 0 < eps <= 1, ell >= 0.5.
 * seeds / gains: host int32[k] / uint64[k] (gains nullable); rep nullable. */
tim_status tim_run(tim_ctx *ctx, const tim_graph *g, int model, int k, double eps, double ell, uint64_t seed,
                   uint32_t flags, int32_t *seeds, uint64_t *gains, tim_report *rep);

/* ---- spread evaluation --------------------------------------------------- */

/* E[I(S)] by forward Monte-Carlo runs, as in the paper's experiments
 * (Section 7) over the live-edge view of Section 2.2.  Run r (runs [first,
 * first+runs)) is the live-edge world of phase 65 and set id r under the
 * rules of the RR sets (IC coins of kind 1 against the thresholds; LT picks of
 * kind 2, with the graph's in-weights if set); its spread is the number of
 * nodes reachable from seeds[0..nseeds) (host int32, repeats allowed) along
 * live edges.  d_counts (device uint32[runs], nullable) receives each run's
 * spread, *total (host, nullable) their sum and *mean (host, nullable) the
 * estimate total / runs.  The first call on a graph builds its out-edge lists
 * (8(n+1) + 8m bytes, freed with the graph). */
tim_status tim_spread_mc(tim_ctx *ctx, const tim_graph *g, int model, uint64_t seed, uint64_t first, uint64_t runs,
                         const int32_t *seeds, int nseeds, uint32_t *d_counts, double *mean, uint64_t *total);

/* ---- batches of queries -------------------------------------------------- */

/* One TIM / TIM+ query of a batch: tim_run's arguments and results. */
typedef struct {
  const tim_graph *graph; /* uploaded to the context passed to tim_run_batch */
  int model;
  int k;
  double eps;
  double ell;
  uint64_t seed;
  uint32_t flags;
  int32_t *seeds;     /* out: host int32[k] */
  uint64_t *gains;    /* out: host uint64[k], or NULL */
  tim_report *report; /* out, or NULL (its times are wall times inside the batch) */
  tim_status status;  /* out: this query's status */
} tim_query;

/* What a batch did. */
typedef struct {
  uint64_t rounds;       /* batched sampling rounds */
  uint64_t jobs;         /* sampling requests served by them */
  uint64_t launches;     /* multi-job launches (one per model, mode and up to 64 requests) */
  uint64_t max_jobs;     /* largest round */
  uint64_t workers;      /* queries run at once */
  uint64_t budget_bytes; /* device memory of the batch */
  uint64_t member_budget_bytes; /* each query's share of it outside NodeSelection */
  double ms_wall;
  double ms_kpt;         /* tim_run_batch: wall time of the device-driven KptEstimation of all queries */
  uint64_t kpt_job_cap;  /* tim_run_batch: most sets a query's job held per KptEstimation step */
  uint64_t kpt_steps;    /* tim_run_batch: device KptEstimation steps run (rounds, launches and jobs above
                            count the batched RefineKPT and NodeSelection requests) */
  uint64_t kpt_graph_launches; /* ... and launches of their captured HIP graph */
  uint64_t rr_pool_bytes;  /* RR pool granted to NodeSelection by the bytes of each query's theta sets */
  uint64_t rr_peak_bytes;  /* most of it granted at once */
  uint64_t held_queries;   /* NodeSelections that waited for memory */
  double held_ms;          /* their waiting time in all */
} tim_batch_info;

/* Runs `count` independent TIM / TIM+ queries (Sections 3.3 and 4.1) at
 * once, at most max_concurrent at a time (0: all).  First, KptEstimation
 * (Algorithm 2) of every query runs on the device with no host step between
 * rounds: a device work queue hands each query chunks of its current round
 * (at most the granularity tim_autotune_batch keeps), persistent multi-query
 * samplers whose wavefronts move from query to query run them, and a device
 * kernel adds each chunk to its round and takes the stop test; these steps
 * are captured in a HIP graph and replayed until every query has stopped.
 * Then each query runs RefineKPT and NodeSelection in a host thread of its
 * own with buffers of its own; the RR sets every query needs at the same
 * point (RefineKPT's sets, NodeSelection's sets) are gathered into one GPU
 * launch whose wavefronts move from query to query as their work runs out.  Each
 * query's seeds, gains and report values other than times and memory
 * figures are those tim_run gives it alone.  The batch's memory is the
 * context's budget less what it holds (without one: 85% of the free device
 * memory); after the large-set slots, each query running at once gets an
 * equal share as its budget, and one whose collection does not fit its
 * share processes it in regenerated chunks, with the same results.  The
 * context's resident-set limit applies to every query.  The graphs must
 * belong to ctx.  Arguments are checked first (TIM_EINVAL, nothing run);
 * then every query runs and the first failing one's status is returned.
 * info (host, nullable) receives the batch's statistics.  The window a
 * round waits for the queries in flight to join it is 1 ms (environment
 * variable TIM_BATCH_WINDOW_US, read per call). */
tim_status tim_run_batch(tim_ctx *ctx, tim_query *queries, int count, int max_concurrent, tim_batch_info *info);

/* What tim_autotune_batch measured and chose. */
typedef struct {
  uint64_t job_cap;   /* the granularity kept: most sets of one query per device KptEstimation step */
  uint64_t caps[4];   /* the candidates: 2^16, 2^18, 2^20, 2^22 */
  double ms_kpt[4];   /* wall time of the batch's device KptEstimation with each (best of 2) */
} tim_batch_tune;

/* Times the device-driven KptEstimation of tim_run_batch on these queries
 * (arguments as for tim_run_batch; nothing is written to their outputs)
 * with each candidate granularity of its work queue - the most sets one
 * query's job holds per step - and keeps the fastest for ctx's later
 * batches if it beats the current one by 3% (default 2^20).  Results of
 * every call do not depend on it.  out (host) may be NULL. */
tim_status tim_autotune_batch(tim_ctx *ctx, tim_query *queries, int count, tim_batch_tune *out);

/* ---- serving: queries that arrive over time ------------------------------ */

typedef struct tim_server tim_server;

/* Starts a request loop on ctx for its resident graphs (upload them first:
 * the large-set slots are sized for the largest).  Up to `slots` queries run
 * at once, each on a member context with an equal share of the context's
 * budget (as in tim_run_batch); the RR-set requests of the queries running
 * at any moment are batched into shared launches, so a query that arrives
 * while others run joins them at the next round.  Further queries wait in
 * a FIFO queue until a slot frees up.  Results are those of tim_run alone.
 * While the server runs, ctx takes no other call but the server's; stop it
 * before destroying ctx. */
tim_status tim_server_start(tim_ctx *ctx, int slots, tim_server **out);

/* Queues one query (arguments as tim_run; TIM_EINVAL if they are invalid).
 * *q and its output arrays must stay valid until tim_server_wait returns for
 * it or the server stops.  *ticket (host) receives its number.  Thread-safe. */
tim_status tim_server_submit(tim_server *srv, tim_query *q, uint64_t *ticket);

/* Blocks until the query of `ticket` is done and returns its status (also
 * in q->status); *latency_ms (host, nullable) receives the time from its
 * submission to its completion.  Thread-safe; may be called more than once. */
tim_status tim_server_wait(tim_server *srv, uint64_t ticket, double *latency_ms);

/* Runs every queued query to completion, stops the threads and frees the
 * server (tickets become invalid).  info (host, nullable) receives the
 * batching statistics of its lifetime. */
tim_status tim_server_stop(tim_server *srv, tim_batch_info *info);

#ifdef __cplusplus
}
#endif

#endif /* TIM_H_ */
