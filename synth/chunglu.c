/*
 * Seeded synthetic input graphs: directed Chung-Lu power-law graphs in
 * canonical in-edge CSR form.
 *
 * This file is an input generator only.  It holds none of the influence
 * maximisation arithmetic (no RR sets, no coin flips, no thresholds): both the
 * HIP path and the CPU oracle consume the arrays it writes as plain data.
 *
 * Definition of the graph produced by synth_chung_lu(n, m, alpha, seed):
 *   - base weights b_i = (i + i0)^(-1/(alpha-1)), i = 0..n-1, with i0 = 1
 *     doubled until the largest expected degree m*b_0/sum(b) is <= n-1;
 *   - the out-weights and the in-weights are two independent Fisher-Yates
 *     permutations of b (uncorrelated in- and out-degree);
 *   - edges are drawn in sequence as (u ~ out-weights, v ~ in-weights) with
 *     Vose alias tables; self-loops are dropped, and of repeated (u,v) pairs
 *     only the first draw is kept; drawing stops at the m-th distinct edge;
 *   - the result is sorted by (dst, src) and returned as in-CSR:
 *     off[v]..off[v+1]-1 are the in-edges of v, src[e] their sources.
 * All random numbers come from one SplitMix64 stream started at `seed`, used
 * in this order: out-permutation, in-permutation, then two words per endpoint
 * of each candidate edge (u first, then v).
 */
#define _POSIX_C_SOURCE 199309L /* clock_gettime under -std=c11 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* Progress lines on stderr for large graphs (synth_set_verbose). */
static int g_verbose = 0;
static struct timespec g_t0;

void synth_set_verbose(int on) { g_verbose = on; }

static void progress(const char *what, int64_t count) {
  if (!g_verbose) return;
  struct timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  double s = (double)(t.tv_sec - g_t0.tv_sec) + 1e-9 * (double)(t.tv_nsec - g_t0.tv_nsec);
  fprintf(stderr, "[synth] %7.1f s  %s %lld\n", s, what, (long long)count);
  fflush(stderr);
}

typedef struct {
  uint64_t key; /* (dst << 32) | src */
  uint64_t idx; /* draw index of the candidate */
} cand_t;

static inline uint64_t sm64_next(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline uint64_t mulhi64(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

/* Vose alias table over weights w[0..n). */
static int build_alias(const double *w, int64_t n, double *prob, int32_t *alias) {
  double sum = 0.0;
  for (int64_t i = 0; i < n; ++i) sum += w[i];
  double *sc = (double *)malloc(sizeof(double) * (size_t)n);
  int64_t *small = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *large = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!sc || !small || !large) { free(sc); free(small); free(large); return -1; }
  int64_t ns = 0, nl = 0;
  for (int64_t i = 0; i < n; ++i) {
    sc[i] = w[i] * (double)n / sum;
    if (sc[i] < 1.0) small[ns++] = i; else large[nl++] = i;
  }
  while (ns > 0 && nl > 0) {
    int64_t s = small[--ns], l = large[--nl];
    prob[s] = sc[s];
    alias[s] = (int32_t)l;
    sc[l] = (sc[l] + sc[s]) - 1.0;
    if (sc[l] < 1.0) small[ns++] = l; else large[nl++] = l;
  }
  while (nl > 0) { int64_t l = large[--nl]; prob[l] = 1.0; alias[l] = (int32_t)l; }
  while (ns > 0) { int64_t s = small[--ns]; prob[s] = 1.0; alias[s] = (int32_t)s; }
  free(sc); free(small); free(large);
  return 0;
}

static inline int32_t alias_draw(uint64_t *st, int64_t n, const double *prob, const int32_t *alias) {
  uint64_t r1 = sm64_next(st), r2 = sm64_next(st);
  int64_t i = (int64_t)mulhi64(r1, (uint64_t)n);
  double u = (double)(r2 >> 11) * 0x1.0p-53;
  return u < prob[i] ? (int32_t)i : alias[i];
}

/* Stable LSD radix sort of a[0..len) on the field selected by `by_idx`
 * (0: key, 1: idx), over the low `bits` bits, 16 bits per pass. */
static int radix_sort(cand_t *a, int64_t len, int by_idx, int bits) {
  cand_t *tmp = (cand_t *)malloc(sizeof(cand_t) * (size_t)(len > 0 ? len : 1));
  int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * 65536);
  if (!tmp || !cnt) { free(tmp); free(cnt); return -1; }
  cand_t *src = a, *dst = tmp;
  for (int shift = 0; shift < bits; shift += 16) {
    memset(cnt, 0, sizeof(int64_t) * 65536);
    for (int64_t i = 0; i < len; ++i) {
      uint64_t f = by_idx ? src[i].idx : src[i].key;
      cnt[(f >> shift) & 0xFFFF]++;
    }
    int64_t run = 0;
    for (int d = 0; d < 65536; ++d) { int64_t c = cnt[d]; cnt[d] = run; run += c; }
    for (int64_t i = 0; i < len; ++i) {
      uint64_t f = by_idx ? src[i].idx : src[i].key;
      dst[cnt[(f >> shift) & 0xFFFF]++] = src[i];
    }
    cand_t *t = src; src = dst; dst = t;
    progress("radix pass done, items", len);
  }
  if (src != a) memcpy(a, src, sizeof(cand_t) * (size_t)len);
  free(tmp); free(cnt);
  return 0;
}

static int bit_length(uint64_t x) { int b = 0; while (x) { ++b; x >>= 1; } return b; }

/*
 * Returns 0 on success, -1 on bad arguments, -2 on allocation failure,
 * -3 if m distinct edges could not be found within 64*m draws.
 * off must hold n+1 entries, src m entries.  realized_i0 may be NULL.
 */
int synth_chung_lu(int64_t n, int64_t m, double alpha, uint64_t seed,
                   int64_t *off, int32_t *src, int64_t *realized_i0) {
  if (n < 2 || n > 0x7FFFFFFF || m < 1 || m > n * (n - 1) || !(alpha > 1.0)) return -1;
  const double beta = 1.0 / (alpha - 1.0);
  clock_gettime(CLOCK_MONOTONIC, &g_t0);
  progress("start: edges wanted", m);
  double *b = (double *)malloc(sizeof(double) * (size_t)n);
  double *wo = (double *)malloc(sizeof(double) * (size_t)n);
  double *wi = (double *)malloc(sizeof(double) * (size_t)n);
  double *po = (double *)malloc(sizeof(double) * (size_t)n);
  double *pi = (double *)malloc(sizeof(double) * (size_t)n);
  int32_t *ao = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *ai = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int rc = 0;
  cand_t *have = NULL, *cand = NULL;
  if (!b || !wo || !wi || !po || !pi || !ao || !ai) { rc = -2; goto done; }

  int64_t i0 = 1;
  for (;;) {
    double sum = 0.0;
    for (int64_t i = 0; i < n; ++i) { b[i] = pow((double)(i + i0), -beta); sum += b[i]; }
    if ((double)m * b[0] / sum <= (double)(n - 1) || i0 > ((int64_t)1 << 40)) break;
    i0 *= 2;
  }
  if (realized_i0) *realized_i0 = i0;

  uint64_t st = seed;
  memcpy(wo, b, sizeof(double) * (size_t)n);
  memcpy(wi, b, sizeof(double) * (size_t)n);
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)mulhi64(sm64_next(&st), (uint64_t)(i + 1));
    double t = wo[i]; wo[i] = wo[j]; wo[j] = t;
  }
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)mulhi64(sm64_next(&st), (uint64_t)(i + 1));
    double t = wi[i]; wi[i] = wi[j]; wi[j] = t;
  }
  if (build_alias(wo, n, po, ao) || build_alias(wi, n, pi, ai)) { rc = -2; goto done; }
  progress("alias tables built, nodes", n);

  const int key_bits = 32 + bit_length((uint64_t)(n - 1));
  have = (cand_t *)malloc(sizeof(cand_t) * (size_t)m);
  if (!have) { rc = -2; goto done; }
  int64_t nhave = 0;
  uint64_t drawn = 0;
  while (nhave < m) {
    int64_t need = m - nhave;
    int64_t batch = need + need / 8 + 1024;
    if (drawn > (uint64_t)m * 64) { rc = -3; goto done; }
    cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)batch);
    if (!cand) { rc = -2; goto done; }
    int64_t nc = 0;
    for (int64_t t = 0; t < batch; ++t) {
      int32_t u = alias_draw(&st, n, po, ao);
      int32_t v = alias_draw(&st, n, pi, ai);
      uint64_t idx = drawn++;
      if ((idx & ((1ull << 28) - 1)) == 0 && idx) progress("candidates drawn so far", (int64_t)idx);
      if (u == v) continue;
      cand[nc].key = ((uint64_t)(uint32_t)v << 32) | (uint32_t)u;
      cand[nc].idx = idx;
      ++nc;
    }
    progress("candidates drawn", nc);
    if (radix_sort(cand, nc, 0, key_bits)) { rc = -2; goto done; }
    /* keep the first draw of every key, then drop keys already kept earlier */
    int64_t nu = 0, h = 0;
    for (int64_t i = 0; i < nc; ++i) {
      if (i > 0 && cand[i].key == cand[i - 1].key) continue;
      while (h < nhave && have[h].key < cand[i].key) ++h;
      if (h < nhave && have[h].key == cand[i].key) continue;
      cand[nu++] = cand[i];
    }
    if (nu > need) {
      /* the last distinct edges drawn fall past the m-th: keep the earliest */
      if (radix_sort(cand, nu, 1, 64)) { rc = -2; goto done; }
      nu = need;
      if (radix_sort(cand, nu, 0, key_bits)) { rc = -2; goto done; }
    }
    /* merge the sorted new keys into `have` from the back */
    int64_t ia = nhave - 1, ib = nu - 1, out = nhave + nu - 1;
    while (ib >= 0) {
      if (ia >= 0 && have[ia].key > cand[ib].key) have[out--] = have[ia--];
      else have[out--] = cand[ib--];
    }
    nhave += nu;
    free(cand); cand = NULL;
    progress("distinct edges kept", nhave);
  }
  memset(off, 0, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t e = 0; e < m; ++e) {
    uint32_t v = (uint32_t)(have[e].key >> 32);
    off[v + 1]++;
    src[e] = (int32_t)(uint32_t)(have[e].key & 0xFFFFFFFFu);
  }
  for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
  progress("in-CSR written, edges", m);

done:
  free(b); free(wo); free(wi); free(po); free(pi); free(ao); free(ai);
  free(have); free(cand);
  return rc;
}
