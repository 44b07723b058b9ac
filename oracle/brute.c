/*
 * Exhaustive checker for the CPU oracle — test infrastructure only.
 *
 * For graphs with at most 24 edges (IC) or a small product of in-degrees
 * (LT), every live-edge world is enumerated with its exact probability, so the
 * quantities the paper's lemmas talk about are computed exactly, with no
 * sampling and without the oracle's random-number stream:
 *   - E[I(S)] for every seed set S (the live-edge view of Section 2.2: the
 *     spread is the expected number of nodes reachable from S when each edge
 *     is kept with its probability);
 *   - Pr[u in R], E[w(R)] and E[kappa(R)] of a random RR set (Definition 2,
 *     Equation (1), Equation (8)).
 * IC edge e is kept with probability (t(e) + 1) / 2^32, the probability that
 * a uniform 32-bit word is <= its uint32 threshold t(e); under the weighted
 * cascade t = floor(2^32/indeg) - 1.  LT: every node of in-degree d >= 1 keeps
 * at most one in-edge: without thresholds each with probability 1/d; with
 * cumulative thresholds t_0 <= .. <= t_{d-1} edge j with probability
 * (t_j - t_{j-1}) / 2^32 (t_{-1} = -1) and none with (2^32 - 1 - t_{d-1}) / 2^32.
 * General triggering (model 2, the explicit distributions of the oracle's
 * reading R11; Section 4.2): node v takes outcome j (its member in-edges are
 * live) with probability (t_j - t_{j-1}) / 2^32, and no in-edge with the rest.
 * For model 2 the thr argument is the address of the distribution (the
 * oracle's orc_trigger layout).
 * Node sets are bit masks, so n <= 20.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAX_TRIG 16 /* outcomes per node, the empty one included */

typedef struct {
  const int64_t *toff;
  const uint32_t *tthr;
  const int64_t *tset;
  const uint32_t *tmem;
} btrigger;

typedef struct {
  int n, m;
  int trig_choices[32];                 /* triggering outcomes at v (0: none) */
  uint64_t trig_live[32][MAX_TRIG];     /* live in-edges of each outcome */
  long double trig_p[32][MAX_TRIG];     /* its probability */
  int eu[64], ev[64]; /* edge e: eu[e] -> ev[e] */
  int indeg[32];
  long double p[64];  /* IC keep probability */
  int first_in[33];   /* in-edges of v are [first_in[v], first_in[v+1]) in CSR order */
  int lt_choices[32];  /* LT: outcomes at v (its in-edges, and the empty set if it has probability) */
  long double lt_p[64 + 32]; /* LT: probability of outcome c of v at lt_p[first_in[v] + v + c] */
} bgraph;

static int load_trigger(bgraph *g, const int64_t *off, const btrigger *tr) {
  for (int v = 0; v < g->n; ++v) {
    int c = 0;
    int64_t prev = -1;
    for (int64_t j = tr->toff[v]; j < tr->toff[v + 1]; ++j) {
      if (c >= MAX_TRIG - 1) return -1;
      uint64_t live = 0;
      for (int64_t i = tr->tset[j]; i < tr->tset[j + 1]; ++i) live |= (uint64_t)1 << (off[v] + tr->tmem[i]);
      g->trig_live[v][c] = live;
      g->trig_p[v][c] = (long double)((int64_t)tr->tthr[j] - prev) / 4294967296.0L;
      prev = (int64_t)tr->tthr[j];
      ++c;
    }
    if (prev < 0xFFFFFFFFLL) {
      g->trig_live[v][c] = 0;
      g->trig_p[v][c] = (long double)(0xFFFFFFFFLL - prev) / 4294967296.0L;
      ++c;
    }
    g->trig_choices[v] = c;
  }
  return 0;
}

static int load(bgraph *g, int64_t n, int64_t m, const int64_t *off, const int32_t *src, const uint32_t *thr,
                int model) {
  if (n < 1 || n > 20 || m < 0 || m > 63) return -1;
  const btrigger *tr = NULL;
  if (model == 2) {
    tr = (const btrigger *)(const void *)thr;
    thr = NULL;
  }
  g->n = (int)n;
  g->m = (int)m;
  for (int v = 0; v < n; ++v) {
    g->first_in[v] = (int)off[v];
    g->indeg[v] = (int)(off[v + 1] - off[v]);
    for (int64_t e = off[v]; e < off[v + 1]; ++e) {
      g->eu[e] = src[e];
      g->ev[e] = v;
      uint64_t t;
      if (thr) t = thr[e];
      else t = (((uint64_t)1 << 32) / (uint64_t)g->indeg[v]) - 1;
      g->p[e] = ((long double)t + 1.0L) / 4294967296.0L;
    }
    /* LT outcomes of v: its in-edges in order, then the empty triggering set */
    const int d = g->indeg[v];
    long double *lp = g->lt_p + off[v] + v;
    g->lt_choices[v] = d;
    if (!thr) {
      for (int j = 0; j < d; ++j) lp[j] = 1.0L / (long double)d;
    } else if (d > 0) {
      int64_t prev = -1;
      for (int j = 0; j < d; ++j) {
        lp[j] = (long double)((int64_t)thr[off[v] + j] - prev) / 4294967296.0L;
        prev = (int64_t)thr[off[v] + j];
      }
      if (prev < 0xFFFFFFFFLL) {
        lp[d] = (long double)(0xFFFFFFFFLL - prev) / 4294967296.0L;
        g->lt_choices[v] = d + 1;
      }
    }
  }
  g->first_in[n] = (int)m;
  if (tr) return load_trigger(g, off, tr);
  return 0;
}

/* Nodes reachable from each node along live edges (reach[u] includes u). */
static void forward_reach(const bgraph *g, uint64_t live, uint32_t *reach) {
  for (int u = 0; u < g->n; ++u) reach[u] = 1u << u;
  int changed = 1;
  while (changed) {
    changed = 0;
    for (int e = 0; e < g->m; ++e) {
      if (!((live >> e) & 1u)) continue;
      /* u -> v live: everything v reaches, u reaches */
      uint32_t before = reach[g->eu[e]];
      uint32_t after = before | reach[g->ev[e]];
      if (after != before) { reach[g->eu[e]] = after; changed = 1; }
    }
  }
}

typedef void (*world_fn)(const bgraph *g, uint64_t live, long double prob, void *ctx);

/* Calls fn once per live-edge world.  Returns the number of worlds, or -1. */
static int64_t for_each_world(const bgraph *g, int model, world_fn fn, void *ctx) {
  if (model == 0) {
    if (g->m > 24) return -1;
    uint64_t worlds = (uint64_t)1 << g->m;
    for (uint64_t live = 0; live < worlds; ++live) {
      long double prob = 1.0L;
      for (int e = 0; e < g->m; ++e) prob *= ((live >> e) & 1u) ? g->p[e] : (1.0L - g->p[e]);
      if (prob == 0.0L) continue;
      fn(g, live, prob, ctx);
    }
    return (int64_t)worlds;
  }
  if (model == 2) {
    /* a mixed-radix counter over the triggering outcome at each node */
    int tc[32];
    int64_t tw = 1;
    for (int v = 0; v < g->n; ++v) {
      tc[v] = 0;
      tw *= g->trig_choices[v];
      if (tw > ((int64_t)1 << 26)) return -1;
    }
    for (int64_t w = 0; w < tw; ++w) {
      uint64_t live = 0;
      long double prob = 1.0L;
      for (int v = 0; v < g->n; ++v) {
        live |= g->trig_live[v][tc[v]];
        prob *= g->trig_p[v][tc[v]];
      }
      if (prob != 0.0L) fn(g, live, prob, ctx);
      for (int v = 0; v < g->n; ++v) {
        if (++tc[v] < g->trig_choices[v]) break;
        tc[v] = 0;
      }
    }
    return tw;
  }
  /* LT: a mixed-radix counter over the outcome at each node (one of its
   * in-edges, or none) */
  int choice[32];
  int64_t worlds = 1;
  for (int v = 0; v < g->n; ++v) {
    choice[v] = 0;
    if (g->lt_choices[v] > 0) worlds *= g->lt_choices[v];
    if (worlds > ((int64_t)1 << 26)) return -1;
  }
  for (int64_t w = 0; w < worlds; ++w) {
    uint64_t live = 0;
    long double prob = 1.0L;
    for (int v = 0; v < g->n; ++v) {
      if (g->lt_choices[v] == 0) continue;
      if (choice[v] < g->indeg[v]) live |= (uint64_t)1 << (g->first_in[v] + choice[v]);
      prob *= g->lt_p[g->first_in[v] + v + choice[v]];
    }
    if (prob != 0.0L) fn(g, live, prob, ctx);
    for (int v = 0; v < g->n; ++v) {
      if (g->lt_choices[v] == 0) continue;
      if (++choice[v] < g->lt_choices[v]) break;
      choice[v] = 0;
    }
  }
  return worlds;
}

/* ---- E[I(S)] for every S ---- */
typedef struct {
  long double *acc; /* 2^n entries */
  uint32_t *reach;
  uint32_t *uni;
} spread_ctx;

static void spread_world(const bgraph *g, uint64_t live, long double prob, void *vctx) {
  spread_ctx *c = (spread_ctx *)vctx;
  forward_reach(g, live, c->reach);
  uint32_t full = 1u << g->n;
  c->uni[0] = 0;
  for (uint32_t mask = 1; mask < full; ++mask) {
    int low = __builtin_ctz(mask);
    c->uni[mask] = c->uni[mask & (mask - 1)] | c->reach[low];
    c->acc[mask] += prob * (long double)__builtin_popcount(c->uni[mask]);
  }
}

int brute_all_spreads(int64_t n, int64_t m, const int64_t *off, const int32_t *src, const uint32_t *thr, int model,
                      double *out) {
  bgraph g;
  if (load(&g, n, m, off, src, thr, model) || n > 16) return -1;
  uint32_t full = 1u << n;
  spread_ctx c;
  c.acc = (long double *)calloc(full, sizeof(long double));
  c.reach = (uint32_t *)calloc(32, sizeof(uint32_t));
  c.uni = (uint32_t *)calloc(full, sizeof(uint32_t));
  if (!c.acc || !c.reach || !c.uni) { free(c.acc); free(c.reach); free(c.uni); return -2; }
  int64_t w = for_each_world(&g, model, spread_world, &c);
  for (uint32_t mask = 0; mask < full; ++mask) out[mask] = (double)c.acc[mask];
  free(c.acc); free(c.reach); free(c.uni);
  return w < 0 ? -1 : 0;
}

/* ---- random RR set statistics ---- */
typedef struct {
  int k;
  long double p_in[32];  /* Pr[u in R] */
  long double ew;        /* E[w(R)] */
  long double ekappa;    /* E[kappa(R)], kappa = 1 - (1 - w/m)^k in long double */
  long double esize;     /* E[|R|] */
  uint32_t reach[32];
} rr_ctx;

static void rr_world(const bgraph *g, uint64_t live, long double prob, void *vctx) {
  rr_ctx *c = (rr_ctx *)vctx;
  forward_reach(g, live, c->reach);
  long double pr = prob / (long double)g->n; /* uniform root */
  for (int root = 0; root < g->n; ++root) {
    /* R = the nodes that reach the root */
    uint32_t r = 0;
    for (int u = 0; u < g->n; ++u)
      if ((c->reach[u] >> root) & 1u) r |= 1u << u;
    long w = 0;
    for (int u = 0; u < g->n; ++u)
      if ((r >> u) & 1u) { c->p_in[u] += pr; w += g->indeg[u]; }
    c->ew += pr * (long double)w;
    c->esize += pr * (long double)__builtin_popcount(r);
    long double q = 1.0L - (long double)w / (long double)g->m;
    c->ekappa += pr * (1.0L - powl(q, (long double)c->k));
  }
}

int brute_rr_stats(int64_t n, int64_t m, const int64_t *off, const int32_t *src, const uint32_t *thr, int model, int k,
                   double *p_in, double *ew, double *ekappa, double *esize) {
  bgraph g;
  if (load(&g, n, m, off, src, thr, model) || m < 1) return -1;
  rr_ctx c;
  memset(&c, 0, sizeof(c));
  c.k = k;
  if (for_each_world(&g, model, rr_world, &c) < 0) return -1;
  for (int u = 0; u < n; ++u) p_in[u] = (double)c.p_in[u];
  *ew = (double)c.ew;
  *ekappa = (double)c.ekappa;
  *esize = (double)c.esize;
  return 0;
}

/* ---- optimum coverage of a set collection by k nodes (n <= 20) ---- */
int64_t brute_max_coverage(int64_t n, uint64_t nsets, const int64_t *set_off, const int32_t *set_nodes, int k,
                           uint32_t *best_mask) {
  if (n > 20 || k < 0) return -1;
  uint32_t *sm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nsets ? nsets : 1));
  if (!sm) return -2;
  for (uint64_t s = 0; s < nsets; ++s) {
    sm[s] = 0;
    for (int64_t i = set_off[s]; i < set_off[s + 1]; ++i) sm[s] |= 1u << set_nodes[i];
  }
  int64_t best = -1;
  uint32_t bm = 0;
  uint32_t full = 1u << n;
  for (uint32_t mask = 0; mask < full; ++mask) {
    if (__builtin_popcount(mask) != k) continue;
    int64_t cov = 0;
    for (uint64_t s = 0; s < nsets; ++s) cov += (sm[s] & mask) != 0;
    if (cov > best) { best = cov; bm = mask; }
  }
  free(sm);
  if (best_mask) *best_mask = bm;
  return best;
}
