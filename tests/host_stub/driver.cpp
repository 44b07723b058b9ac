// Drives the host side of batches and servers (api.cpp built against the
// stand-in runtime) from many threads at once, for ThreadSanitizer and
// AddressSanitizer builds.  Every query of a batch and every served query
// must equal the same query run alone.  Test support only.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "tim.h"

namespace {

struct Csr {
  int64_t n = 0, m = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> src;
  std::vector<uint32_t> thr;
};

Csr random_graph(int64_t n, int64_t m, unsigned seed) {
  std::mt19937_64 r(seed);
  std::vector<std::pair<int32_t, int32_t>> e;  // (dst, src)
  while ((int64_t)e.size() < m * 2) {
    const int32_t u = (int32_t)(r() % (uint64_t)n), v = (int32_t)(r() % (uint64_t)n);
    if (u != v) e.emplace_back(v, u);
  }
  std::sort(e.begin(), e.end());
  e.erase(std::unique(e.begin(), e.end()), e.end());
  e.resize((size_t)std::min<int64_t>(m, (int64_t)e.size()));
  std::sort(e.begin(), e.end());
  Csr g;
  g.n = n;
  g.m = (int64_t)e.size();
  g.off.assign((size_t)n + 1, 0);
  for (auto& x : e) g.off[(size_t)x.first + 1]++;
  for (int64_t v = 0; v < n; ++v) g.off[(size_t)v + 1] += g.off[(size_t)v];
  for (auto& x : e) g.src.push_back(x.second);
  for (int64_t i = 0; i < g.m; ++i) g.thr.push_back((uint32_t)(r() >> 32));
  return g;
}

struct Result {
  std::vector<int32_t> seeds;
  std::vector<uint64_t> gains;
  tim_report rep;
};

void check(tim_status st, const char* what) {
  if (st != TIM_OK) {
    fprintf(stderr, "%s failed: %d %s\n", what, (int)st, tim_last_error());
    exit(2);
  }
}

bool same(const Result& a, const Result& b) {
  return a.seeds == b.seeds && a.gains == b.gains && a.rep.kpt.i_last == b.rep.kpt.i_last &&
         a.rep.kpt.kpt_star == b.rep.kpt.kpt_star && a.rep.refine.kpt_plus == b.rep.refine.kpt_plus &&
         a.rep.select.theta == b.rep.select.theta && a.rep.select.nodes == b.rep.select.nodes;
}

}  // namespace

int main(int argc, char** argv) {
  const int rounds = argc > 1 ? atoi(argv[1]) : 2;
  const uint64_t budget = argc > 2 ? strtoull(argv[2], nullptr, 10) : 0;
  const int nq = argc > 3 ? atoi(argv[3]) : 24;
  tim_ctx* ctx = nullptr;
  check(tim_ctx_create(0, nullptr, budget, &ctx), "tim_ctx_create");
  std::vector<Csr> gs = {random_graph(3000, 12000, 1), random_graph(800, 5000, 2), random_graph(5000, 15000, 3)};
  std::vector<tim_graph*> dg;
  for (size_t i = 0; i < gs.size(); ++i) {
    tim_graph* g = nullptr;
    check(tim_graph_upload(ctx, gs[i].n, gs[i].m, gs[i].off.data(), gs[i].src.data(),
                           i == 1 ? gs[i].thr.data() : nullptr, &g),
          "tim_graph_upload");
    dg.push_back(g);
  }
  // queries: graph, model, k, eps
  std::mt19937 r(7);
  std::vector<tim_query> qs((size_t)nq);
  std::vector<Result> alone((size_t)nq), got((size_t)nq);
  for (int i = 0; i < nq; ++i) {
    const int gi = (int)(r() % gs.size());
    const int k = 1 + (int)(r() % 12);
    qs[(size_t)i] = tim_query{dg[(size_t)gi], (int)(r() % 2), k, 0.3 + 0.1 * (r() % 5), 1.0, 100u + (unsigned)i, 0u,
                              nullptr, nullptr, nullptr, TIM_OK};
    Result& a = alone[(size_t)i];
    a.seeds.assign((size_t)k, 0);
    a.gains.assign((size_t)k, 0);
    check(tim_run(ctx, qs[(size_t)i].graph, qs[(size_t)i].model, k, qs[(size_t)i].eps, 1.0, qs[(size_t)i].seed, 0,
                  a.seeds.data(), a.gains.data(), &a.rep),
          "tim_run");
  }
  auto bind = [&](int i) {
    Result& g = got[(size_t)i];
    g.seeds.assign((size_t)qs[(size_t)i].k, -1);
    g.gains.assign((size_t)qs[(size_t)i].k, 0);
    memset(&g.rep, 0, sizeof(g.rep));
    qs[(size_t)i].seeds = g.seeds.data();
    qs[(size_t)i].gains = g.gains.data();
    qs[(size_t)i].report = &g.rep;
  };
  for (int round = 0; round < rounds; ++round) {
    // a batch with 16 workers
    for (int i = 0; i < nq; ++i) bind(i);
    tim_batch_info info;
    check(tim_run_batch(ctx, qs.data(), nq, 16, &info), "tim_run_batch");
    for (int i = 0; i < nq; ++i)
      if (!same(got[(size_t)i], alone[(size_t)i])) {
        fprintf(stderr, "batch query %d differs from its run alone\n", i);
        return 3;
      }
    // a server with 8 slots and 3 submitting threads
    for (int i = 0; i < nq; ++i) bind(i);
    tim_server* srv = nullptr;
    check(tim_server_start(ctx, 8, &srv), "tim_server_start");
    std::vector<uint64_t> tickets((size_t)nq);
    std::vector<std::thread> subs;
    for (int t = 0; t < 3; ++t)
      subs.emplace_back([&, t] {
        for (int i = t; i < nq; i += 3) check(tim_server_submit(srv, &qs[(size_t)i], &tickets[(size_t)i]), "submit");
      });
    for (auto& th : subs) th.join();
    std::vector<std::thread> waiters;
    for (int t = 0; t < 2; ++t)
      waiters.emplace_back([&, t] {
        for (int i = t; i < nq; i += 2) {
          double ms = 0;
          check(tim_server_wait(srv, tickets[(size_t)i], &ms), "wait");
        }
      });
    for (auto& th : waiters) th.join();
    check(tim_server_stop(srv, &info), "tim_server_stop");
    for (int i = 0; i < nq; ++i)
      if (!same(got[(size_t)i], alone[(size_t)i])) {
        fprintf(stderr, "served query %d differs from its run alone\n", i);
        return 4;
      }
    printf("round %d: batch and server ok (held %llu)\n", round, (unsigned long long)info.held_queries);
    fflush(stdout);
  }
  for (tim_graph* g : dg) tim_graph_free(g);
  tim_ctx_destroy(ctx);
  printf("done\n");
  return 0;
}
