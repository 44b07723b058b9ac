/*
 * CPU ORACLE for TIM / TIM+ — test infrastructure, not part of the product.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this code.  It shares no source with the HIP path: it has its own Philox,
 * its own RR-set search, its own greedy and its own scalar formulas, written
 * plainly and single-threaded (compile with -O2 -ffp-contract=off, no
 * fast-math).
 *
 * Paper: Tang, Xiao, Shi, "Influence Maximization: Near-Optimal Time
 * Complexity Meets Practical Efficiency", SIGMOD 2014.
 *
 * What is computed, and where the paper defines it:
 *   - random RR set: Definitions 1-2 (Section 2.3); built by the randomized
 *     reverse BFS of Section 3.1 (its implementation paragraph) for IC and by the
 *     triggering-set BFS of Section 4.2 for LT (one in-edge per node, the
 *     LT-as-triggering description of Section 7.1);
 *   - width w(R): Equation (1);  kappa(R): Equation (8), Lemma 5;
 *   - KptEstimation: Algorithm 2, with c_i from Equation (9);
 *   - greedy maximum coverage: Algorithm 1, and its use on R' in Algorithm 3;
 *   - RefineKPT: Algorithm 3 with the epsilon' of Section 4.1;
 *   - lambda: Equation (4);  TIM: Section 3.3;  TIM+: Section 4.1.
 *
 * Where the paper leaves a choice open, this file follows the readings below
 * (the HIP path follows the same readings, implemented separately):
 *   R1 random numbers: Philox4x32-10 (Salmon et al., SC'11).  key = (seed lo,
 *      seed hi); counter = (idx lo, phase<<24 | kind<<16 | (idx>>32 & 0xFFFF),
 *      set lo, set hi).  kind 0 = root (idx 0), 1 = IC coin group (idx = e>>2,
 *      output word e&3), 2 = LT pick (idx = node), 3 = triggering-set pick
 *      (idx = node, reading R11).  phase i in [1,62] =
 *      KptEstimation round i, 63 = RefineKPT's fresh sets, 64 = NodeSelection.
 *   R2 an IC edge e is live iff its 32-bit word x satisfies x <= t(e), where
 *      t(e) = floor(p(e) * 2^32) - 1 is the edge's uint32 threshold; under the
 *      weighted cascade p = 1/indeg(v) and t = floor(2^32 / indeg(v)) - 1.
 *   R3 root = floor(X64 * n / 2^64), X64 = word1<<32 | word0 of the root draw.
 *   R4 LT pick at node v: j = floor(X64 * indeg(v) / 2^64), in-edge off[v]+j;
 *      the walk stops at a node of in-degree 0 or at an already visited node.
 *   R9 LT with in-weights (Section 7.1: random weights normalized per node)
 *      is given as per-edge uint32 cumulative thresholds t_0 <= .. <= t_{d-1}
 *      over v's in-edges in CSR order: t_j = floor(C_j * 2^32) - 1 for the
 *      cumulative weight C_j.  With x = word0 of the pick draw at v, the walk
 *      takes the first in-edge j with x <= t_j, and stops at v if x > t_{d-1}
 *      (the empty triggering set, of probability 1 - C_{d-1}).  Edge j has
 *      probability (t_j - t_{j-1}) / 2^32 with t_{-1} = -1.
 *  R10 spread evaluation (the live-edge view of Section 2.2; Monte-Carlo runs
 *      as in the paper's experiments, Section 7): run r uses the live-edge
 *      world of phase 65 and set id r, with the coins and picks of R2, R4,
 *      R9 and R11.  Its spread is the number of nodes reachable from S along live
 *      edges (S included); E[I(S)] is estimated by the mean over runs.
 *  R11 general triggering model (Section 4.2): each node v draws its
 *      triggering set T(v), a subset of its in-neighbours, from a distribution
 *      given explicitly as outcomes j in [toff[v], toff[v+1]) with uint32
 *      cumulative thresholds tthr[j] (t_j = floor(C_j * 2^32) - 1 for the
 *      cumulative probability C_j, non-decreasing within v) and members
 *      tmem[tset[j] .. tset[j+1]): local in-edge indices i (the in-edge
 *      off[v] + i), increasing within an outcome.  With x = word0 of the draw
 *      of kind 3 at (phase, set, idx = v), T(v) is the first outcome with
 *      x <= t_j, and empty if there is none (probability 1 - C_last).  The RR
 *      set is the randomized BFS of Section 4.2: every dequeued node draws its
 *      T(v) and its unvisited members are queued.  Entry points take, for
 *      model 2, the address of an orc_trigger in place of their thr argument.
 *   R5 kappa in IEEE binary64 without contraction: q = 1 - w/m, r = q^k by
 *      binary exponentiation (r=1,b=q; per bit: if set r*=b; shift; if more
 *      bits b*=b), kappa = 1 - r.  kappa*2^53 is an integer; the round sum is
 *      the exact 128-bit integer S = sum(kappa * 2^53).
 *   R6 rounds i = 1 .. floor(log2 n) - 1; c_i = ceil(a * 2^i) with
 *      a = 6*ell*ln(n) + 6*ln(log2 n); stop iff S * 2^i > c_i * 2^53;
 *      KPT* = ((double)S * 2^-53 * n) / (2 * c_i); KPT* = 1 if no round stops.
 *   R7 greedy: the node of largest count among the unselected, ties to the
 *      lowest id; always k distinct nodes.
 *   R8 scalars in binary64 with the evaluation order written below; the
 *      numbers of sets are ceilings.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, written from the SC'11 definition.                          */
/* ------------------------------------------------------------------------- */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 = k0 + 0x9E3779B9u; /* Weyl increment: golden ratio */
      k1 = k1 + 0xBB67AE85u; /* Weyl increment: sqrt(3) - 1 */
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ x1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ x3 ^ k1;
    uint32_t n3 = lo0;
    x0 = n0; x1 = n1; x2 = n2; x3 = n3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One Philox output block for (seed, phase, kind, idx, set) per reading R1. */
void orc_draw(uint64_t seed, uint32_t phase, uint32_t kind, uint64_t idx, uint64_t set, uint32_t out[4]) {
  uint32_t ctr[4], key[2];
  ctr[0] = (uint32_t)(idx & 0xFFFFFFFFu);
  ctr[1] = (phase << 24) | (kind << 16) | (uint32_t)((idx >> 32) & 0xFFFFu);
  ctr[2] = (uint32_t)(set & 0xFFFFFFFFu);
  ctr[3] = (uint32_t)(set >> 32);
  key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
  key[1] = (uint32_t)(seed >> 32);
  orc_philox4x32_10(ctr, key, out);
}

/* Uniform root of a random RR set (Definition 2; reading R3). */
int64_t orc_root(uint64_t seed, uint32_t phase, uint64_t set, int64_t n) {
  uint32_t x[4];
  orc_draw(seed, phase, 0, 0, set, x);
  uint64_t x64 = ((uint64_t)x[1] << 32) | x[0];
  return (int64_t)(((u128)x64 * (u128)(uint64_t)n) >> 64);
}

/* The 32-bit word that decides IC edge e (reading R1). */
uint32_t orc_coin_word(uint64_t seed, uint32_t phase, uint64_t set, int64_t e) {
  uint32_t x[4];
  orc_draw(seed, phase, 1, (uint64_t)e >> 2, set, x);
  return x[e & 3];
}

/* Weighted-cascade threshold of an edge into a node of in-degree d >= 1 (R2). */
uint32_t orc_wc_threshold(int64_t d) {
  uint64_t t = ((uint64_t)1 << 32) / (uint64_t)d; /* floor(2^32 / d) */
  return (uint32_t)(t - 1);
}

/* LT pick at a node of in-degree d >= 1: index j in [0, d) (reading R4). */
int64_t orc_lt_pick(uint64_t seed, uint32_t phase, uint64_t set, int64_t v, int64_t d) {
  uint32_t x[4];
  orc_draw(seed, phase, 2, (uint64_t)v, set, x);
  uint64_t x64 = ((uint64_t)x[1] << 32) | x[0];
  return (int64_t)(((u128)x64 * (u128)(uint64_t)d) >> 64);
}

/* LT pick with cumulative thresholds t[0..d) at node v (reading R9): the
 * index of the in-edge taken, or -1 if the walk stops at v. */
int64_t orc_lt_pick_cumulative(uint64_t seed, uint32_t phase, uint64_t set, int64_t v, const uint32_t *t,
                               int64_t d) {
  uint32_t x[4];
  orc_draw(seed, phase, 2, (uint64_t)v, set, x);
  for (int64_t j = 0; j < d; ++j)
    if (x[0] <= t[j]) return j;
  return -1;
}

/* The triggering distribution of reading R11. */
typedef struct {
  const int64_t *toff;  /* n+1 */
  const uint32_t *tthr; /* one per outcome */
  const int64_t *tset;  /* outcomes + 1 */
  const uint32_t *tmem; /* local in-edge indices */
} orc_trigger;

/* Outcome drawn at node v under reading R11 (an index into tthr / tset), or
 * -1 for the empty triggering set. */
int64_t orc_trig_pick(uint64_t seed, uint32_t phase, uint64_t set, int64_t v, const int64_t *toff,
                      const uint32_t *tthr) {
  uint32_t x[4];
  orc_draw(seed, phase, 3, (uint64_t)v, set, x);
  for (int64_t j = toff[v]; j < toff[v + 1]; ++j)
    if (x[0] <= tthr[j]) return j;
  return -1;
}

/* ------------------------------------------------------------------------- */
/* Graph and per-set workspace.                                              */
/* ------------------------------------------------------------------------- */

typedef struct {
  int64_t n, m;
  const int64_t *off;  /* in-CSR offsets, n+1 */
  const int32_t *src;  /* sources of in-edges, sorted by (dst, src) */
  const uint32_t *thr; /* per-edge thresholds of the model: IC live thresholds (NULL: weighted
                          cascade), LT cumulative thresholds (NULL: uniform 1/indeg) */
} orc_graph;

typedef struct {
  int64_t n;
  uint32_t *mark;  /* visited stamps */
  uint32_t stamp;
  int32_t *queue;  /* BFS queue = the RR set's nodes */
} orc_ws;

static orc_ws *ws_new(int64_t n) {
  orc_ws *w = (orc_ws *)calloc(1, sizeof(orc_ws));
  if (!w) return NULL;
  w->n = n;
  w->mark = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
  w->queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!w->mark || !w->queue) { free(w->mark); free(w->queue); free(w); return NULL; }
  return w;
}

static void ws_free(orc_ws *w) {
  if (!w) return;
  free(w->mark); free(w->queue); free(w);
}

static void ws_next_stamp(orc_ws *w) {
  if (w->stamp == 0xFFFFFFFFu) {
    memset(w->mark, 0, sizeof(uint32_t) * (size_t)w->n);
    w->stamp = 0;
  }
  w->stamp++;
}

static int edge_is_live(const orc_graph *g, uint64_t seed, uint32_t phase, uint64_t set, int64_t e,
                        int64_t indeg_of_dst) {
  uint32_t x = orc_coin_word(seed, phase, set, e);
  uint32_t t = g->thr ? g->thr[e] : orc_wc_threshold(indeg_of_dst);
  return x <= t;
}

/*
 * One random RR set (IC: randomized reverse BFS over in-edges; LT: reverse
 * walk along the one live in-edge of each node).  The set's nodes are left in
 * w->queue[0..return value); *width receives w(R) = sum of in-degrees.
 */
static int64_t rr_set(const orc_graph *g, int model, uint64_t seed, uint32_t phase, uint64_t set, orc_ws *w,
                      uint64_t *width) {
  ws_next_stamp(w);
  int64_t root = orc_root(seed, phase, set, g->n);
  w->mark[root] = w->stamp;
  w->queue[0] = (int32_t)root;
  int64_t len = 1;
  uint64_t wsum = 0;
  if (model == 0) {
    int64_t head = 0;
    while (head < len) {
      int64_t v = w->queue[head++];
      int64_t a = g->off[v], b = g->off[v + 1];
      wsum += (uint64_t)(b - a);
      for (int64_t e = a; e < b; ++e) {
        int32_t u = g->src[e];
        if (w->mark[u] == w->stamp) continue;
        if (edge_is_live(g, seed, phase, set, e, b - a)) {
          w->mark[u] = w->stamp;
          w->queue[len++] = u;
        }
      }
    }
  } else if (model == 2) {
    const orc_trigger *tr = (const orc_trigger *)(const void *)g->thr;
    int64_t head = 0;
    while (head < len) {
      int64_t v = w->queue[head++];
      int64_t a = g->off[v];
      wsum += (uint64_t)(g->off[v + 1] - a);
      int64_t j = orc_trig_pick(seed, phase, set, v, tr->toff, tr->tthr);
      if (j < 0) continue;
      for (int64_t i = tr->tset[j]; i < tr->tset[j + 1]; ++i) {
        int32_t u = g->src[a + tr->tmem[i]];
        if (w->mark[u] == w->stamp) continue;
        w->mark[u] = w->stamp;
        w->queue[len++] = u;
      }
    }
  } else {
    int64_t v = root;
    for (;;) {
      int64_t a = g->off[v], d = g->off[v + 1] - a;
      wsum += (uint64_t)d;
      if (d == 0) break;
      int64_t j = g->thr ? orc_lt_pick_cumulative(seed, phase, set, v, g->thr + a, d)
                         : orc_lt_pick(seed, phase, set, v, d);
      if (j < 0) break; /* the empty triggering set */
      int32_t u = g->src[a + j];
      if (w->mark[u] == w->stamp) break;
      w->mark[u] = w->stamp;
      w->queue[len++] = u;
      v = u;
    }
  }
  *width = wsum;
  return len;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/*
 * Sets [first, first+count) of (seed, phase): node lists sorted ascending into
 * nodes[] (capacity cap) with offsets set_off[0..count], widths into widths[]
 * (may be NULL).  Returns the total number of nodes, -1 if cap is too small,
 * -2 on allocation failure.
 */
int64_t orc_sample_sets(int64_t n, int64_t m, const int64_t *off, const int32_t *src, const uint32_t *thr, int model,
                        uint64_t seed, uint32_t phase, uint64_t first, uint64_t count, int64_t *set_off,
                        int32_t *nodes, int64_t cap, uint64_t *widths) {
  orc_graph g = {n, m, off, src, thr};
  orc_ws *w = ws_new(n);
  if (!w) return -2;
  int64_t total = 0;
  set_off[0] = 0;
  for (uint64_t s = 0; s < count; ++s) {
    uint64_t wd;
    int64_t len = rr_set(&g, model, seed, phase, first + s, w, &wd);
    if (total + len > cap) { ws_free(w); return -1; }
    memcpy(nodes + total, w->queue, sizeof(int32_t) * (size_t)len);
    qsort(nodes + total, (size_t)len, sizeof(int32_t), cmp_i32);
    total += len;
    set_off[s + 1] = total;
    if (widths) widths[s] = wd;
  }
  ws_free(w);
  return total;
}

/* ------------------------------------------------------------------------- */
/* kappa (Equation (8)) and the scalar formulas.                             */
/* ------------------------------------------------------------------------- */

double orc_kappa(uint64_t w, int64_t m, int k) {
  double q = 1.0 - (double)w / (double)m;
  double r = 1.0, b = q;
  unsigned int e = (unsigned int)k;
  while (e) {
    if (e & 1u) r = r * b;
    e >>= 1;
    if (e) b = b * b;
  }
  return 1.0 - r;
}

/* kappa * 2^53 as an integer (exact: kappa is a multiple of 2^-53 in [0,1]). */
uint64_t orc_kappa_fixed(uint64_t w, int64_t m, int k) {
  return (uint64_t)ldexp(orc_kappa(w, m, k), 53);
}

double orc_ln_binom(int64_t n, int k) {
  double s = 0.0;
  for (int i = 0; i < k; ++i) s = s + (log((double)(n - i)) - log((double)(i + 1)));
  return s;
}

/* Equation (4). */
double orc_lambda(int64_t n, int k, double eps, double ell) {
  double nd = (double)n;
  return ((8.0 + 2.0 * eps) * nd * ((ell * log(nd) + orc_ln_binom(n, k)) + log(2.0))) / (eps * eps);
}

/* epsilon' of Section 4.1. */
double orc_eps_prime(int k, double eps, double ell) {
  return 5.0 * cbrt(ell * eps * eps / ((double)k + ell));
}

/* lambda' of Algorithm 3. */
double orc_lambda_prime(int64_t n, double eps_p, double ell) {
  double nd = (double)n;
  return ((2.0 + eps_p) * ell * nd * log(nd)) / (eps_p * eps_p);
}

/* Number of rounds of Algorithm 2: floor(log2 n) - 1 (reading R6). */
int orc_i_max(int64_t n) {
  int bits = 0;
  uint64_t x = (uint64_t)n;
  while (x) { ++bits; x >>= 1; }
  return bits - 2;
}

/* c_i of Equation (9), rounded up (reading R6). */
uint64_t orc_c_i(int64_t n, double ell, int i) {
  double nd = (double)n;
  double a = 6.0 * ell * log(nd) + 6.0 * log(log2(nd));
  return (uint64_t)ceil(ldexp(a, i));
}

/* ------------------------------------------------------------------------- */
/* Greedy maximum coverage (Algorithm 1; the greedy on R' in Algorithm 3).   */
/* ------------------------------------------------------------------------- */

int orc_greedy(int64_t n, uint64_t nsets, const int64_t *set_off, const int32_t *set_nodes, int k, int32_t *seeds,
               uint64_t *gains) {
  int64_t total = nsets ? set_off[nsets] : 0;
  int64_t *cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int64_t *inv_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t *cursor = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  uint64_t *inv = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(total > 0 ? total : 1));
  char *covered = (char *)calloc((size_t)(nsets > 0 ? nsets : 1), 1);
  char *selected = (char *)calloc((size_t)n, 1);
  if (!cnt || !inv_off || !cursor || !inv || !covered || !selected) {
    free(cnt); free(inv_off); free(cursor); free(inv); free(covered); free(selected);
    return -2;
  }
  /* coverage count of each node and the node -> sets index */
  for (int64_t i = 0; i < total; ++i) cnt[set_nodes[i]]++;
  for (int64_t u = 0; u < n; ++u) inv_off[u + 1] = inv_off[u] + cnt[u];
  for (int64_t u = 0; u < n; ++u) cursor[u] = inv_off[u];
  for (uint64_t s = 0; s < nsets; ++s)
    for (int64_t i = set_off[s]; i < set_off[s + 1]; ++i) inv[cursor[set_nodes[i]]++] = s;

  for (int j = 0; j < k; ++j) {
    int64_t best = -1;
    for (int64_t u = 0; u < n; ++u) {
      if (selected[u]) continue;
      if (best < 0 || cnt[u] > cnt[best]) best = u;
    }
    seeds[j] = (int32_t)best;
    gains[j] = (uint64_t)cnt[best];
    selected[best] = 1;
    for (int64_t i = inv_off[best]; i < inv_off[best + 1]; ++i) {
      uint64_t s = inv[i];
      if (covered[s]) continue;
      covered[s] = 1;
      for (int64_t t = set_off[s]; t < set_off[s + 1]; ++t) cnt[set_nodes[t]]--;
    }
  }
  free(cnt); free(inv_off); free(cursor); free(inv); free(covered); free(selected);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* The three phases and the TIM / TIM+ drivers.                              */
/* ------------------------------------------------------------------------- */

#define ORC_MAX_ROUNDS 64

typedef struct {
  /* KptEstimation (Algorithm 2) */
  int32_t i_max, i_last;
  uint64_t c_last;
  double kpt_star;
  uint64_t round_c[ORC_MAX_ROUNDS];
  uint64_t round_sum_lo[ORC_MAX_ROUNDS], round_sum_hi[ORC_MAX_ROUNDS];
  uint64_t round_width[ORC_MAX_ROUNDS], round_nodes[ORC_MAX_ROUNDS];
  /* RefineKPT (Algorithm 3) */
  double eps_prime, lambda_prime, kpt_prime, kpt_plus;
  uint64_t theta_prime, covered_prime;
  /* NodeSelection (Algorithm 1) */
  double lambda, ell_used;
  uint64_t theta, ns_nodes, ns_width, ns_covered;
} orc_report;

static int valid_graph(const orc_graph *g) {
  if (g->n < 2 || g->m < 1 || !g->off || !g->src) return 0;
  if (g->off[0] != 0 || g->off[g->n] != g->m) return 0;
  return 1;
}

/* One round of Algorithm 2 (its c_i sets and their kappa sum): sets
 * [first, first+count) of phase `phase`, the exact sum of kappa(R) * 2^53
 * (Equation (8)) and the widths and sizes of the sets. */
static void round_sum(const orc_graph *g, int model, uint64_t seed, uint32_t phase, uint64_t first, uint64_t count,
                      int k, orc_ws *w, u128 *sum, uint64_t *wsum, uint64_t *nsum) {
  *sum = 0;
  *wsum = 0;
  *nsum = 0;
  for (uint64_t s = first; s < first + count; ++s) {
    uint64_t wd;
    int64_t len = rr_set(g, model, seed, phase, s, w, &wd);
    *sum += orc_kappa_fixed(wd, g->m, k);
    *wsum += wd;
    *nsum += (uint64_t)len;
  }
}

/* round_sum over a range of set ids: out = {S low, S high, width, size}. */
int orc_round_sum(int64_t n, int64_t m, const int64_t *off, const int32_t *src, const uint32_t *thr, int model,
                  uint64_t seed, uint32_t phase, uint64_t first, uint64_t count, int k, uint64_t out[4]) {
  orc_graph g = {n, m, off, src, thr};
  if (!valid_graph(&g) || k < 1) return -1;
  orc_ws *w = ws_new(n);
  if (!w) return -2;
  u128 sum;
  round_sum(&g, model, seed, phase, first, count, k, w, &sum, &out[2], &out[3]);
  out[0] = (uint64_t)sum;
  out[1] = (uint64_t)(sum >> 64);
  ws_free(w);
  return 0;
}

int orc_kpt_estimate(int64_t n, int64_t m, const int64_t *off, const int32_t *src, const uint32_t *thr, int model,
                     uint64_t seed, int k, double ell, orc_report *rep) {
  orc_graph g = {n, m, off, src, thr};
  if (!valid_graph(&g) || k < 1 || k > n) return -1;
  orc_ws *w = ws_new(n);
  if (!w) return -2;
  int imax = orc_i_max(n);
  rep->i_max = imax;
  rep->kpt_star = 1.0;
  rep->i_last = imax;
  rep->c_last = imax >= 1 ? orc_c_i(n, ell, imax) : 0;
  for (int i = 1; i <= imax; ++i) {
    uint64_t ci = orc_c_i(n, ell, i);
    u128 sum;
    uint64_t wsum, nsum;
    round_sum(&g, model, seed, (uint32_t)i, 0, ci, k, w, &sum, &wsum, &nsum);
    rep->round_c[i] = ci;
    rep->round_sum_lo[i] = (uint64_t)sum;
    rep->round_sum_hi[i] = (uint64_t)(sum >> 64);
    rep->round_width[i] = wsum;
    rep->round_nodes[i] = nsum;
    /* sum/c_i > 2^-i  <=>  S * 2^i > c_i * 2^53  (S = sum * 2^53, exact) */
    int stop = (sum << i) > ((u128)ci << 53);
    if (stop) {
      double sum_d = ldexp((double)sum, -53);
      rep->kpt_star = (sum_d * (double)n) / (2.0 * (double)ci);
      rep->i_last = i;
      rep->c_last = ci;
      break;
    }
  }
  ws_free(w);
  return 0;
}

static int collect_sets(const orc_graph *g, int model, uint64_t seed, uint32_t phase, uint64_t count,
                        int64_t **set_off_out, int32_t **nodes_out, uint64_t *width_total) {
  orc_ws *w = ws_new(g->n);
  int64_t *so = (int64_t *)malloc(sizeof(int64_t) * (size_t)(count + 1));
  int64_t cap = 1024;
  int32_t *nodes = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
  if (!w || !so || !nodes) { ws_free(w); free(so); free(nodes); return -2; }
  int64_t total = 0;
  uint64_t wt = 0;
  so[0] = 0;
  for (uint64_t s = 0; s < count; ++s) {
    uint64_t wd;
    int64_t len = rr_set(g, model, seed, phase, s, w, &wd);
    if (total + len > cap) {
      while (total + len > cap) cap *= 2;
      int32_t *nn = (int32_t *)realloc(nodes, sizeof(int32_t) * (size_t)cap);
      if (!nn) { ws_free(w); free(so); free(nodes); return -2; }
      nodes = nn;
    }
    memcpy(nodes + total, w->queue, sizeof(int32_t) * (size_t)len);
    total += len;
    so[s + 1] = total;
    wt += wd;
  }
  ws_free(w);
  *set_off_out = so;
  *nodes_out = nodes;
  if (width_total) *width_total = wt;
  return 0;
}

int orc_refine_kpt(int64_t n, int64_t m, const int64_t *off, const int32_t *src, const uint32_t *thr, int model,
                   uint64_t seed, int k, double eps, double ell, double kpt_star, int i_last, uint64_t c_last,
                   int32_t *s_prime, orc_report *rep) {
  orc_graph g = {n, m, off, src, thr};
  if (!valid_graph(&g) || k < 1 || k > n || !(eps > 0.0 && eps <= 1.0)) return -1;
  /* S'_k: greedy on the sets of the last round of Algorithm 2 */
  int64_t *so = NULL;
  int32_t *nodes = NULL;
  int rc = collect_sets(&g, model, seed, (uint32_t)i_last, c_last, &so, &nodes, NULL);
  if (rc) return rc;
  uint64_t *gains = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)k);
  if (!gains) { free(so); free(nodes); return -2; }
  rc = orc_greedy(n, c_last, so, nodes, k, s_prime, gains);
  free(so); free(nodes); free(gains);
  if (rc) return rc;
  /* eps', lambda', theta': fresh sets, fraction covered by S'_k */
  double eps_p = orc_eps_prime(k, eps, ell);
  double lambda_p = orc_lambda_prime(n, eps_p, ell);
  uint64_t theta_p = (uint64_t)ceil(lambda_p / kpt_star);
  char *in_s = (char *)calloc((size_t)n, 1);
  orc_ws *w = ws_new(n);
  if (!in_s || !w) { free(in_s); ws_free(w); return -2; }
  for (int j = 0; j < k; ++j) in_s[s_prime[j]] = 1;
  uint64_t hit = 0;
  for (uint64_t s = 0; s < theta_p; ++s) {
    uint64_t wd;
    int64_t len = rr_set(&g, model, seed, 63u, s, w, &wd);
    for (int64_t i = 0; i < len; ++i) {
      if (in_s[w->queue[i]]) { ++hit; break; }
    }
  }
  free(in_s); ws_free(w);
  /* KPT' from that fraction, and KPT+ */
  double f = (double)hit / (double)theta_p;
  double kpt_p = f * (double)n / (1.0 + eps_p);
  rep->eps_prime = eps_p;
  rep->lambda_prime = lambda_p;
  rep->theta_prime = theta_p;
  rep->covered_prime = hit;
  rep->kpt_prime = kpt_p;
  rep->kpt_plus = kpt_p > kpt_star ? kpt_p : kpt_star;
  return 0;
}

int orc_node_select(int64_t n, int64_t m, const int64_t *off, const int32_t *src, const uint32_t *thr, int model,
                    uint64_t seed, int k, uint64_t theta, int32_t *seeds, uint64_t *gains, orc_report *rep) {
  orc_graph g = {n, m, off, src, thr};
  if (!valid_graph(&g) || k < 1 || k > n) return -1;
  int64_t *so = NULL;
  int32_t *nodes = NULL;
  uint64_t wt = 0;
  int rc = collect_sets(&g, model, seed, 64u, theta, &so, &nodes, &wt);
  if (rc) return rc;
  rc = orc_greedy(n, theta, so, nodes, k, seeds, gains);
  rep->theta = theta;
  rep->ns_nodes = theta ? (uint64_t)so[theta] : 0;
  rep->ns_width = wt;
  uint64_t cov = 0;
  for (int j = 0; j < k; ++j) cov += gains[j];
  rep->ns_covered = cov;
  free(so); free(nodes);
  return rc;
}

/* flags: bit 0 = plain TIM (no RefineKPT); bit 1 = scale ell for 1 - n^-ell overall success. */
int orc_tim_run(int64_t n, int64_t m, const int64_t *off, const int32_t *src, const uint32_t *thr, int model, int k,
                double eps, double ell, uint64_t seed, uint32_t flags, int32_t *seeds, uint64_t *gains,
                int32_t *s_prime, orc_report *rep) {
  if (n < 2 || m < 1 || k < 1 || k > n || !(eps > 0.0 && eps <= 1.0) || !(ell >= 0.5)) return -1;
  memset(rep, 0, sizeof(*rep));
  int plain = (flags & 1u) != 0;
  double ell_used = ell;
  if (flags & 2u) ell_used = ell * (1.0 + log(plain ? 2.0 : 3.0) / log((double)n));
  rep->ell_used = ell_used;
  int rc = orc_kpt_estimate(n, m, off, src, thr, model, seed, k, ell_used, rep);
  if (rc) return rc;
  double lb = rep->kpt_star;
  if (!plain) {
    rc = orc_refine_kpt(n, m, off, src, thr, model, seed, k, eps, ell_used, rep->kpt_star, rep->i_last, rep->c_last,
                        s_prime, rep);
    if (rc) return rc;
    lb = rep->kpt_plus;
  }
  rep->lambda = orc_lambda(n, k, eps, ell_used);
  uint64_t theta = (uint64_t)ceil(rep->lambda / lb);
  return orc_node_select(n, m, off, src, thr, model, seed, k, theta, seeds, gains, rep);
}

/* Width of set `set` and whether it meets the node set marked in `in_s`. */
int64_t orc_rr_single(int64_t n, int64_t m, const int64_t *off, const int32_t *src, const uint32_t *thr, int model,
                      uint64_t seed, uint32_t phase, uint64_t set, int32_t *nodes_out, uint64_t *width) {
  orc_graph g = {n, m, off, src, thr};
  orc_ws *w = ws_new(n);
  if (!w) return -2;
  int64_t len = rr_set(&g, model, seed, phase, set, w, width);
  memcpy(nodes_out, w->queue, sizeof(int32_t) * (size_t)len);
  qsort(nodes_out, (size_t)len, sizeof(int32_t), cmp_i32);
  ws_free(w);
  return len;
}

size_t orc_report_size(void) { return sizeof(orc_report); }

/* ------------------------------------------------------------------------- */
/* Spread evaluation by forward Monte-Carlo runs (reading R10).              */
/* ------------------------------------------------------------------------- */

enum { ORC_PHASE_EVAL = 65 };

/* Is in-edge e of v (in-degree d, first in-edge a) live in world (seed, phase, run)? */
static int edge_live_in_world(const orc_graph *g, int model, uint64_t seed, uint32_t phase, uint64_t run,
                              int64_t v, int64_t a, int64_t d, int64_t e) {
  if (model == 0) return edge_is_live(g, seed, phase, run, e, d);
  if (model == 2) {
    const orc_trigger *tr = (const orc_trigger *)(const void *)g->thr;
    int64_t jt = orc_trig_pick(seed, phase, run, v, tr->toff, tr->tthr);
    if (jt < 0) return 0;
    for (int64_t i = tr->tset[jt]; i < tr->tset[jt + 1]; ++i)
      if (a + (int64_t)tr->tmem[i] == e) return 1;
    return 0;
  }
  int64_t j = g->thr ? orc_lt_pick_cumulative(seed, phase, run, v, g->thr + a, d) : orc_lt_pick(seed, phase, run, v, d);
  return j >= 0 && a + j == e;
}

/*
 * Runs [first, first+count): counts[i] = number of nodes reachable from the
 * seed set in the world of run first+i.  Returns 0, or -1 on a bad seed and
 * -2 on allocation failure.
 */
int orc_forward_spread(int64_t n, int64_t m, const int64_t *off, const int32_t *src, const uint32_t *thr, int model,
                       uint64_t seed, uint64_t first, uint64_t count, const int32_t *seeds, int nseeds,
                       uint64_t *counts) {
  orc_graph g = {n, m, off, src, thr};
  /* out-edges: for each source u, the in-edge ids e with src[e] == u */
  int64_t *out_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t *out_e = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
  int64_t *dst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  orc_ws *w = ws_new(n);
  if (!out_off || !out_e || !dst || !fill || !w) {
    free(out_off); free(out_e); free(dst); free(fill); ws_free(w);
    return -2;
  }
  for (int64_t v = 0; v < n; ++v)
    for (int64_t e = off[v]; e < off[v + 1]; ++e) {
      out_off[src[e] + 1]++;
      dst[e] = v;
    }
  for (int64_t u = 0; u < n; ++u) out_off[u + 1] += out_off[u];
  for (int64_t u = 0; u < n; ++u) fill[u] = out_off[u];
  for (int64_t e = 0; e < m; ++e) out_e[fill[src[e]]++] = e;
  int rc = 0;
  for (int i = 0; i < nseeds; ++i)
    if (seeds[i] < 0 || seeds[i] >= n) rc = -1;
  for (uint64_t r = 0; r < count && rc == 0; ++r) {
    const uint64_t run = first + r;
    ws_next_stamp(w);
    int64_t len = 0;
    for (int i = 0; i < nseeds; ++i) {
      if (w->mark[seeds[i]] == w->stamp) continue;
      w->mark[seeds[i]] = w->stamp;
      w->queue[len++] = seeds[i];
    }
    for (int64_t head = 0; head < len; ++head) {
      int64_t u = w->queue[head];
      for (int64_t x = out_off[u]; x < out_off[u + 1]; ++x) {
        int64_t e = out_e[x], v = dst[e];
        if (w->mark[v] == w->stamp) continue;
        int64_t a = off[v], d = off[v + 1] - a;
        if (edge_live_in_world(&g, model, seed, ORC_PHASE_EVAL, run, v, a, d, e)) {
          w->mark[v] = w->stamp;
          w->queue[len++] = (int32_t)v;
        }
      }
    }
    counts[r] = (uint64_t)len;
  }
  free(out_off); free(out_e); free(dst); free(fill); ws_free(w);
  return rc;
}
