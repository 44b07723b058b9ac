// Runs the same queries (tim_run) on contexts with device-memory budgets from
// a geometric sweep, on the CPU build of api.cpp against the stand-in runtime.
// A larger budget must never turn a success into a failure: from the
// smallest budget at which every query succeeds on, every query must succeed
// with the results of the run without a budget.  Prints one line per budget.
// Test support only.
#include <algorithm>
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "tim.h"

namespace {

struct Csr {
  int64_t n = 0, m = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> src;
};

// n nodes, each with `deg` distinct random in-neighbours (sorted by source)
Csr ring_graph(int64_t n, int deg, unsigned seed) {
  std::mt19937_64 r(seed);
  Csr g;
  g.n = n;
  g.off.push_back(0);
  for (int64_t v = 0; v < n; ++v) {
    std::vector<int32_t> in;
    while ((int)in.size() < deg) {
      const int32_t u = (int32_t)(r() % (uint64_t)n);
      bool dup = u == v;
      for (int32_t x : in) dup = dup || x == u;
      if (!dup) in.push_back(u);
    }
    std::sort(in.begin(), in.end());
    for (int32_t u : in) g.src.push_back(u);
    g.off.push_back((int64_t)g.src.size());
  }
  g.m = (int64_t)g.src.size();
  return g;
}

struct Query {
  int graph, model, k;
  double eps;
  uint64_t seed;
};

struct Result {
  tim_status st = TIM_OK;
  std::vector<int32_t> seeds;
  std::vector<uint64_t> gains;
  tim_report rep;
};

bool same(const Result& a, const Result& b) {
  return a.seeds == b.seeds && a.gains == b.gains && a.rep.kpt.i_last == b.rep.kpt.i_last &&
         a.rep.kpt.kpt_star == b.rep.kpt.kpt_star && a.rep.refine.kpt_plus == b.rep.refine.kpt_plus &&
         a.rep.refine.covered_prime == b.rep.refine.covered_prime && a.rep.select.theta == b.rep.select.theta &&
         a.rep.select.nodes == b.rep.select.nodes && a.rep.select.width == b.rep.select.width;
}

void print_diff(size_t q, const Result& a, const Result& b) {
  printf("  query %zu: seeds %s gains %s i_last %d/%d kpt_star %.17g/%.17g kpt_plus %.17g/%.17g covered' %" PRIu64
         "/%" PRIu64 " theta %" PRIu64 "/%" PRIu64 " nodes %" PRIu64 "/%" PRIu64 " width %" PRIu64 "/%" PRIu64 "\n",
         q, a.seeds == b.seeds ? "same" : "differ", a.gains == b.gains ? "same" : "differ", a.rep.kpt.i_last,
         b.rep.kpt.i_last, a.rep.kpt.kpt_star, b.rep.kpt.kpt_star, a.rep.refine.kpt_plus, b.rep.refine.kpt_plus,
         a.rep.refine.covered_prime, b.rep.refine.covered_prime, a.rep.select.theta, b.rep.select.theta,
         a.rep.select.nodes, b.rep.select.nodes, a.rep.select.width, b.rep.select.width);
}

std::vector<Result> run_all(uint64_t budget, const std::vector<Csr>& gs, const std::vector<Query>& qs,
                            std::vector<std::string>* errors) {
  tim_ctx* ctx = nullptr;
  std::vector<Result> out(qs.size());
  if (tim_ctx_create(0, nullptr, budget, &ctx) != TIM_OK) {
    fprintf(stderr, "tim_ctx_create failed: %s\n", tim_last_error());
    exit(2);
  }
  std::vector<tim_graph*> dg;
  for (const Csr& g : gs) {
    tim_graph* h = nullptr;
    if (tim_graph_upload(ctx, g.n, g.m, g.off.data(), g.src.data(), nullptr, &h) != TIM_OK) {
      fprintf(stderr, "tim_graph_upload failed: %s\n", tim_last_error());
      exit(2);
    }
    dg.push_back(h);
  }
  for (size_t i = 0; i < qs.size(); ++i) {
    const Query& q = qs[i];
    Result& r = out[i];
    r.seeds.assign((size_t)q.k, -1);
    r.gains.assign((size_t)q.k, 0);
    memset(&r.rep, 0, sizeof(r.rep));
    r.st = tim_run(ctx, dg[(size_t)q.graph], q.model, q.k, q.eps, 1.0, q.seed, 0, r.seeds.data(), r.gains.data(),
                   &r.rep);
    if (r.st != TIM_OK && errors) errors->push_back("query " + std::to_string(i) + ": " + tim_last_error());
  }
  for (tim_graph* h : dg) tim_graph_free(h);
  tim_ctx_destroy(ctx);
  return out;
}

}  // namespace

int main(int argc, char** argv) {
  const uint64_t lo = argc > 1 ? strtoull(argv[1], nullptr, 10) : (1u << 18);
  const uint64_t hi = argc > 2 ? strtoull(argv[2], nullptr, 10) : (1u << 28);
  const double step = argc > 3 ? atof(argv[3]) : 1.2;
  const std::vector<Csr> gs = {ring_graph(3000, 4, 1), ring_graph(800, 6, 2)};
  const std::vector<Query> qs = {{0, 0, 5, 0.3, 11}, {0, 1, 1, 0.5, 12}, {1, 0, 8, 0.4, 13}, {1, 1, 3, 0.3, 14}};
  const std::vector<Result> ref = run_all(0, gs, qs, nullptr);
  for (size_t i = 0; i < qs.size(); ++i)
    if (ref[i].st != TIM_OK) {
      fprintf(stderr, "query %zu fails without a budget: %s\n", i, tim_last_error());
      return 2;
    }
  bool all_ok_seen = false;
  int bad = 0;
  for (double b = (double)lo; b <= (double)hi; b *= step) {
    const uint64_t budget = (uint64_t)b;
    std::vector<std::string> errors;
    const std::vector<Result> got = run_all(budget, gs, qs, &errors);
    int ok = 0, differ = 0;
    for (size_t i = 0; i < qs.size(); ++i) {
      if (got[i].st != TIM_OK) continue;
      ++ok;
      if (!same(got[i], ref[i])) ++differ;
    }
    for (size_t i = 0; i < qs.size(); ++i)
      if (got[i].st == TIM_OK && !same(got[i], ref[i])) print_diff(i, got[i], ref[i]);
    printf("budget %" PRIu64 ": %d of %zu ok, %d differ%s%s\n", budget, ok, qs.size(), differ,
           errors.empty() ? "" : "; first error: ", errors.empty() ? "" : errors[0].c_str());
    if (differ) ++bad;
    if (ok == (int)qs.size()) all_ok_seen = true;
    else if (all_ok_seen) ++bad;  // a larger budget than one that ran everything failed a query
  }
  if (!all_ok_seen) {
    printf("no budget of the sweep ran every query\n");
    return 3;
  }
  printf(bad ? "FAILED: %d budgets\n" : "done\n", bad);
  return bad ? 4 : 0;
}
