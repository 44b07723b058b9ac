// Stand-in "kernels" for the CPU build of the host driver: each launch runs
// at once on the calling thread (or is recorded while its stream is
// captured) and writes what the real kernels report - counters, widths, set
// records and node lists, argmax keys - for stand-in RR sets derived from
// the keys (seed, phase, set id), so that every host path of api.cpp runs.
// They compute no step of the method faithfully.  Test support only.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "engine.hpp"
#include "host_stub.h"

namespace tim {
namespace {

typedef unsigned __int128 u128;

uint64_t mix(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Most nodes of a stand-in set.
constexpr int kStubMaxSet = 512;

// With TIM_STUB_GROWTH=1 the sets of KptEstimation round i have up to 2^i
// nodes (at most 256), so that each round's sets are about twice the size of
// the previous round's; with TIM_STUB_GROWTH=2 the sets of RefineKPT and
// NodeSelection have up to 512 nodes besides.  Otherwise every set has 1-3
// nodes.
int stand_in_cap(uint32_t phase) {
  static const int growth = [] {
    const char* e = getenv("TIM_STUB_GROWTH");
    return e ? atoi(e) : 0;
  }();
  if (growth >= 2 && phase > 62) return kStubMaxSet;
  if (growth < 1 || phase < 1 || phase > 62) return 3;
  return phase >= 8 ? 256 : std::max(3, 1 << phase);
}

// A stand-in set of distinct nodes and its width.
int stand_in_set(const SampleArgs& a, uint64_t id, int32_t* nodes, uint64_t* width) {
  const uint64_t h = mix(a.seed ^ ((uint64_t)a.phase << 40) ^ mix(id));
  const int cap = stand_in_cap(a.phase);
  int len = 1 + (int)(h % (uint64_t)cap);
  if (len > a.g.n) len = (int)a.g.n;
  *width = std::min<uint64_t>((uint64_t)a.g.m, 1 + (h >> 16) % 12);
  if (cap > 3) {
    // consecutive node ids from a random start: distinct while len <= n
    const uint64_t start = mix(h) % (uint64_t)a.g.n;
    for (int j = 0; j < len; ++j) nodes[j] = (int32_t)((start + (uint64_t)j) % (uint64_t)a.g.n);
    return len;
  }
  int got = 0;
  for (int j = 0; got < len && j < 16; ++j) {
    const int32_t v = (int32_t)(mix(h + (uint64_t)j) % (uint64_t)a.g.n);
    bool dup = false;
    for (int t = 0; t < got; ++t) dup = dup || nodes[t] == v;
    if (!dup) nodes[got++] = v;
  }
  return got;
}

uint64_t kappa_fixed(uint64_t w, int64_t m, int k) {
  const double q = 1.0 - (double)w / (double)m;
  double r = 1.0, b = q;
  for (unsigned e = (unsigned)k; e; e >>= 1) {
    if (e & 1u) r *= b;
    if (e > 1u) b *= b;
  }
  return (uint64_t)std::ldexp(1.0 - r, 53);
}

void run_sample(int model, int mode, const SampleArgs& a) {
  (void)model;
  unsigned long long* c = a.ctr;
  unsigned long long* acc = c + kCtrAcc;
  u128 kap = 0;
  int32_t nodes[kStubMaxSet];
  for (uint64_t i = 0; i < a.count; ++i) {
    uint64_t w = 0;
    const int len = stand_in_set(a, a.first + i, nodes, &w);
    acc[kAccWidth] += w;
    acc[kAccNodes] += (unsigned long long)len;
    if (mode == kModeWidth) {
      a.wbuf[i] = (uint32_t)w;
      if (a.sizes) a.sizes[i] = (uint32_t)len;
      kap += kappa_fixed(w, a.g.m, a.k);
    } else if (mode == kModeEmit) {
      const unsigned long long pos = c[kCtrPoolCursor];
      c[kCtrPoolCursor] += (unsigned long long)len;
      if (pos + (unsigned long long)len <= a.pool_cap)
        for (int t = 0; t < len; ++t) a.pool[pos + (unsigned long long)t] = nodes[t];
      a.set_start[i] = a.pool_base + pos;
      a.set_len[i] = (uint32_t)len;
      if (a.widths) a.widths[i] = w;
      if (a.wbuf) {
        a.wbuf[i] = (uint32_t)w;
        kap += kappa_fixed(w, a.g.m, a.k);
      }
    } else {
      bool hit = false;
      for (int t = 0; t < len; ++t) hit = hit || ((a.seed_bits[(uint32_t)nodes[t] >> 5] >> (nodes[t] & 31)) & 1u);
      if (hit) acc[kAccCovered] += 1;
    }
  }
  const u128 old = ((u128)acc[kAccKappaHi] << 64) | (u128)acc[kAccKappaLo];
  const u128 sum = old + kap;
  acc[kAccKappaLo] = (unsigned long long)sum;
  acc[kAccKappaHi] = (unsigned long long)(sum >> 64);
}

void set_keys(unsigned long long* best, int k) {
  for (int j = 0; j < k; ++j) best[j] = 0xFFFFFFFFull - (unsigned long long)j;
}

void* g_scratch = nullptr;
std::mutex g_scratch_mu;

}  // namespace

void launch_clear_counters(unsigned long long* ctr, hipStream_t s) {
  stub_submit(s, [=] { memset(ctr, 0, kCtrCount * sizeof(unsigned long long)); });
}
int ic_seg_lanes() { return 8; }
int ic_blocks_per_cu(int, bool, int) { return 4; }
int ic_tier1_blocks_per_cu(int, bool) { return 2; }
int lt_lane_blocks_per_cu(int) { return 4; }
int trig_blocks_per_cu(int) { return 4; }
int trig_tier1_blocks_per_cu(int) { return 4; }
int lt_chain_blocks_per_cu(int, bool) { return 2; }
uint32_t tier0_set_cap(int model, int seg_lanes) {
  if (model == 1) return 64;
  if (model == 2) return 256;
  return seg_lanes <= 8 ? 128u : 512u;
}
void launch_sample(int model, int mode, const SampleArgs& a, int, int, int, hipStream_t s, hipEvent_t) {
  stub_submit(s, [=] { run_sample(model, mode, a); });
}
int batch_blocks_per_cu(int, int, bool, int) { return 4; }
void launch_clear_counters_batch(const JobTable& t, hipStream_t s) {
  stub_submit(s, [=] {
    for (int j = 0; j < t.njobs; ++j) memset(t.jobs[j].ctr, 0, kCtrCount * sizeof(unsigned long long));
  });
}
void launch_sample_batch(int model, int mode, bool, const JobTable& t, int, int, int, uint64_t, hipStream_t s,
                         hipEvent_t) {
  stub_submit(s, [=] {
    for (int j = 0; j < t.njobs; ++j) run_sample(model, mode, t.jobs[j]);
  });
}

void launch_kpt_jobs(const KptStepArgs& a, hipStream_t s) {
  stub_submit(s, [=] {
    uint64_t used = 0;
    for (int j = 0; j < a.nq; ++j) {
      const KptQuery& q = a.q[j];
      SampleArgs x = SampleArgs();
      x.g = q.g;
      x.seed = q.seed;
      x.k = q.k;
      x.ctr = a.ctr + (size_t)j * kCtrCount;
      x.wbuf = a.wbuf + used;
      x.list1 = a.list1 + used;
      x.list2 = a.list2 ? a.list2 + used : nullptr;
      if (q.round > 0 && !q.err) {
        const uint64_t left = q.c[q.round] - q.pos;
        uint64_t take = std::min(left, a.job_cap);
        take = std::min(take, a.step_cap - used);
        x.phase = (uint32_t)q.round;
        x.first = q.pos;
        x.count = take;
        used += take;
      }
      a.jobs[j] = x;
    }
  });
}

void launch_kpt_advance(const KptStepArgs& a, hipStream_t s) {
  stub_submit(s, [=] {
    *a.active = 0;
    for (int j = 0; j < a.nq; ++j) {
      KptQuery& q = a.q[j];
      const SampleArgs& x = a.jobs[j];
      if (q.round > 0 && x.count > 0) {
        u128 sum = ((u128)q.sum_hi << 64) | (u128)q.sum_lo;
        const unsigned long long* acc = x.ctr + kCtrAcc;
        sum += ((u128)acc[kAccKappaHi] << 64) | (u128)acc[kAccKappaLo];
        q.width += acc[kAccWidth];
        q.nodes += acc[kAccNodes];
        q.sum_lo = (unsigned long long)sum;
        q.sum_hi = (unsigned long long)(sum >> 64);
        q.pos += x.count;
        const int i = q.round;
        if (q.pos == q.c[i]) {
          q.r_lo[i] = q.sum_lo;
          q.r_hi[i] = q.sum_hi;
          q.r_width[i] = q.width;
          q.r_nodes[i] = q.nodes;
          if ((sum << i) > ((u128)q.c[i] << 53)) {
            q.i_last = i;
            q.round = 0;
          } else if (i >= q.imax) {
            q.i_last = q.imax;
            q.round = 0;
          } else {
            q.round = i + 1;
            q.pos = 0;
            q.sum_lo = q.sum_hi = q.width = q.nodes = 0;
          }
        }
      }
      if (q.round > 0 && !q.err) *a.active += 1;
    }
  });
}

void launch_out_csr_count(const int32_t* src, int64_t m, uint32_t* cnt, hipStream_t s) {
  stub_submit(s, [=] {
    for (int64_t e = 0; e < m; ++e) cnt[src[e]] += 1;
  });
}
void launch_out_csr_scatter(const int64_t*, const int32_t*, int64_t, int64_t, const int64_t*, uint32_t*, int32_t*,
                            uint32_t*, hipStream_t) {}
void launch_spread(int, const SpreadArgs& a, hipStream_t s) {
  stub_submit(s, [=] {
    a.ctr[0] = a.runs;
    a.ctr[1] = a.runs * (unsigned long long)a.nseeds;
  });
}

size_t scan_temp_bytes(uint64_t len) { return (len / 4096 + 2) * 8; }
size_t bucket_workspace_bytes(int64_t n, uint64_t total, bool index) { return 256 + (size_t)n / 64 + total * (index ? 8 : 4); }
void launch_scan_u32_to_i64(const uint32_t* in, int64_t* out, uint64_t len, void*, hipStream_t s) {
  stub_submit(s, [=] {
    int64_t acc = 0;
    for (uint64_t i = 0; i < len; ++i) {
      out[i] = acc;
      acc += in[i];
    }
    out[len] = acc;
  });
}
void launch_compact(const int32_t* pool, const uint64_t* set_start, const uint32_t* set_len, const int64_t* out_off,
                    int32_t* out_nodes, uint64_t nsets, hipStream_t s) {
  stub_submit(s, [=] {
    for (uint64_t i = 0; i < nsets; ++i)
      memcpy(out_nodes + out_off[i], pool + set_start[i], set_len[i] * sizeof(int32_t));
  });
}
void launch_check_ids(const int32_t* nodes, uint64_t total, int64_t n, unsigned int* flag, hipStream_t s) {
  stub_submit(s, [=] {
    *flag = 0;
    for (uint64_t i = 0; i < total; ++i)
      if (nodes[i] < 0 || nodes[i] >= n) *flag = 1;
  });
}
void launch_set_sizes(const int64_t* set_off, uint32_t* sizes, uint64_t nsets, hipStream_t s) {
  stub_submit(s, [=] {
    for (uint64_t i = 0; i < nsets; ++i) sizes[i] = (uint32_t)(set_off[i + 1] - set_off[i]);
  });
}
void launch_counts(const GreedyArgs& a, hipStream_t s) {
  stub_submit(s, [=] { memset(a.cnt, 0, (size_t)a.n * 4); });
}
void launch_index(const GreedyArgs& a, hipStream_t s) { launch_counts(a, s); }
void launch_greedy(const GreedyArgs& a, int k, hipStream_t s) {
  stub_submit(s, [=] { set_keys(a.best, k); });
}
void launch_zero_counts(uint32_t* cnt, int64_t n, hipStream_t s) {
  stub_submit(s, [=] { memset(cnt, 0, (size_t)n * 4); });
}
void launch_greedy_init(const GreedyArgs& a, uint64_t covered_len, int k, hipStream_t s) {
  stub_submit(s, [=] {
    if (covered_len) memset(a.covered, 0, covered_len);
    memset(a.selected, 0, (size_t)a.n);
    memset(a.best, 0, (size_t)k * 8);
  });
}
void launch_argmax_step(const GreedyArgs& a, int j, hipStream_t s) {
  stub_submit(s, [=] { a.best[j] = 0xFFFFFFFFull - (unsigned long long)j; });
}
void launch_cover_step(const GreedyArgs&, int, hipStream_t) {}
void launch_pool_hist(const int32_t* pool, const uint64_t* set_start, const uint32_t* set_len, uint64_t nsets,
                      uint32_t* cnt, hipStream_t s) {
  stub_submit(s, [=] {
    for (uint64_t i = 0; i < nsets; ++i)
      for (uint32_t t = 0; t < set_len[i]; ++t) cnt[pool[set_start[i] + t]] += 1;
  });
}
void launch_pool_cover(const unsigned long long*, const int32_t*, const uint64_t*, const uint32_t*, uint64_t,
                       uint8_t*, uint32_t*, hipStream_t) {}

size_t static_scratch_bytes() { return (size_t)64 << 20; }
hipError_t static_scratch_init(int) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch) g_scratch = calloc(1, static_scratch_bytes());
  return g_scratch ? hipSuccess : hipErrorOutOfMemory;
}
StaticGreedy static_greedy_layout(int) {
  StaticGreedy st;
  memset(&st, 0, sizeof(st));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  unsigned char* b = static_cast<unsigned char*>(g_scratch);
  if (!b) return st;
  st.cnt = reinterpret_cast<uint32_t*>(b);
  st.fill = reinterpret_cast<uint32_t*>(b + (4u << 20));
  st.inv_off = reinterpret_cast<int64_t*>(b + (8u << 20));
  st.inv_sets = reinterpret_cast<uint32_t*>(b + (20u << 20));
  st.covered = b + (40u << 20);
  st.selected = b + (48u << 20);
  st.best = reinterpret_cast<unsigned long long*>(b + (50u << 20));
  st.flag = reinterpret_cast<unsigned int*>(b + (51u << 20));
  st.zero_off = reinterpret_cast<int64_t*>(b + (51u << 20) + 64);
  st.scan_temp = b + (52u << 20);
  return st;
}
void launch_set_u64(unsigned long long* p, unsigned long long v, hipStream_t s) {
  stub_submit(s, [=] { *p = v; });
}

}  // namespace tim
