// Host driver of the TIM / TIM+ engine: the C ABI declared in include/tim.h.
//
// The phases follow the paper: KptEstimation (Algorithm 2), RefineKPT
// (Algorithm 3) and NodeSelection (Algorithm 1), assembled as TIM
// (Section 3.3) and TIM+ (Section 4.1).  Every RR set is produced on the GPU
// by the samplers in sample.hip and every coverage step by coverage.hip; the
// host only evaluates the scalar formulas (Equations (4) and (9), epsilon',
// lambda', theta', KPT', KPT+) in binary64 with a fixed evaluation order, and
// reads back per-launch totals.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.hpp"
#include "tim.h"

using tim::SampleArgs;

namespace {

typedef unsigned __int128 u128;

thread_local std::string g_error;

tim_status fail(tim_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(TIM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define TIM_TRY(expr)                  \
  do {                                 \
    tim_status s_ = (expr);            \
    if (s_ != TIM_OK) return s_;       \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// Sets per sampling launch: bounds the deferred-set list of one launch.
constexpr uint64_t kMaxLaunchSets = 1ull << 26;

// Algorithmic bytes per visited node of the general triggering model: its
// two CSR offsets (16), its two outcome offsets (16), one outcome threshold
// (4), the outcome's two member offsets (16), and the member and source that
// brought it in (8).
constexpr uint64_t kTriggerNodeBytes = 60;

struct Hub;

}  // namespace

struct tim_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint64_t budget = 0;
  uint64_t held = 0;
  int num_cu = 0;
  int seg_lanes = 8;
  uint32_t slice_cap = tim::kPoolChunk;  // largest node-pool slice of a wavefront
  uint32_t slice_cap_set = tim::kPoolChunk;  // its value outside the chunked plan (tim_autotune may change it)
  uint32_t emit_wave_sets = 0;           // emit launches: at least this many sets per tier-0 wavefront
  uint32_t slice = tim::kPoolChunk;      // slice of the current emit launches
  uint64_t resident_limit = ~0ull;       // most sets a greedy keeps resident
  int emit_kappa_k = 0;                  // emit launches also sum kappa(R) for this k (0: no)
  // the node pool holds the sets of one KptEstimation round (Algorithm 3 reuses them as R')
  struct Stored {
    bool valid = false;
    const void* graph = nullptr;
    int model = 0;
    uint64_t seed = 0, count = 0, nodes = 0, width = 0;
    uint32_t phase = 0;
  } stored;
  int grid_ic[3][2] = {};
  int grid_ic64[3][2] = {};
  int grid_ic_wide[3][2] = {};  // first tier with 64 lanes per set (launches of few sets)
  bool wide_small = true;       // launches of few sets take the 64-lane shape (off while tim_autotune times shapes)
  int grid_lt[3] = {};
  int grid_lt_chain[3] = {};
  int grid_trig[3] = {};          // general-triggering first tier
  int grid_trig1[3] = {};         // general-triggering one-set-per-wavefront tier
  int grid_rounds[2][2] = {};     // multi-job launches of KptEstimation rounds: tier 0 per [model][wc]
  int grid_batch1[2] = {};        // their IC tier 1, per wc
  int grid_batch_chain = 0;       // their LT long-chain tier
  DevBuf jobs;                    // job table and per-job counters of a multi-job launch
  unsigned long long* ctr = nullptr;       // device counters of the current launch
  unsigned long long* ctr_host = nullptr;  // pinned mirror
  DevBuf list1, list2, wbuf, pool, set_start, set_len;
  DevBuf big_stamp, big_queue, big_epoch;
  int big_slots = 0;
  int64_t big_n = -1;
  DevBuf rr_off, rr_nodes, sizes, cnt, fill, inv_off, inv_sets, covered, selected, best, scan_tmp, seed_bits;
  DevBuf bucket;  // the greedy's counting sort by node range (tim::bucket_workspace_bytes)
  hipEvent_t ev[2] = {nullptr, nullptr};
  // batch member: its sampling launches go to the hub
  Hub* hub = nullptr;
  const tim_ctx* parent = nullptr;  // whose graphs it may use
  uint64_t share = 0;               // its budget outside NodeSelection (the rest comes from the hub's RR pool)
  // batches run on this context: the hub and its member contexts, kept
  // (with their buffers) from one tim_run_batch call to the next
  Hub* batch = nullptr;
  std::vector<tim_ctx*> members;
  bool serving = false;  // a server runs on this context
  uint64_t batch_job_cap = 1ull << 20;  // sets a query's job holds per step of the batch's device KptEstimation
  int64_t max_graph_n = 0;  // largest graph uploaded to this context
  hipEvent_t ready_ev = nullptr;
  bool prof_on = false;
  hipEvent_t pev[3] = {nullptr, nullptr, nullptr};
  tim_profile prof = {};
};

struct tim_graph {
  tim_ctx* ctx = nullptr;
  int64_t n = 0, m = 0;
  int64_t* off = nullptr;
  uint32_t* off32 = nullptr;  // the offsets in 32 bits (m < 2^32): one 8-byte read gives a node's in-list range
  int32_t* src = nullptr;
  uint32_t* thr = nullptr;
  uint32_t* lthr = nullptr;  // LT cumulative in-weight thresholds, or nullptr (1/indeg)
  // general triggering model: explicit per-node distributions over in-edge subsets (or none)
  int64_t* toff = nullptr;
  uint32_t* tthr = nullptr;
  int64_t* tset = nullptr;
  uint32_t* tmem = nullptr;
  // out-edge lists for the spread evaluator, built on first use
  int64_t* out_off = nullptr;
  int32_t* out_dst = nullptr;
  uint32_t* out_eid = nullptr;
};

namespace {

tim_status ensure(tim_ctx* c, DevBuf& b, size_t bytes, const char* what) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return TIM_OK;
  size_t want = std::max(bytes, b.bytes + b.bytes / 2);
  want = (want + 255) & ~(size_t)255;
  const uint64_t others = c->held - b.bytes;
  if (c->budget && others + want > c->budget) {
    want = (bytes + 255) & ~(size_t)255;
    if (others + want > c->budget)
      return fail(TIM_EBUDGET, "%s needs %zu bytes; %llu of the %llu-byte budget are in use", what, bytes,
                  (unsigned long long)others, (unsigned long long)c->budget);
  }
  if (b.p) {
    (void)hipStreamSynchronize(c->stream);  // kernels in flight may still read it
    (void)hipFree(b.p);
  }
  c->held = others;
  b.p = nullptr;
  b.bytes = 0;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();  // the failed allocation is reported here, not by the next launch check
    return fail(TIM_ENOMEM, "hipMalloc of %zu bytes for %s failed", want, what);
  }
  b.bytes = want;
  c->held += want;
  return TIM_OK;
}

void release(tim_ctx* c, DevBuf& b) {
  if (b.p) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(b.p);
  }
  c->held -= b.bytes;
  b = DevBuf();
}

tim_graph const* check_graph(const tim_ctx* c, const tim_graph* g) {
  return (c && g && (g->ctx == c || (c->parent && g->ctx == c->parent))) ? g : nullptr;
}

// Per-slot visited stamps and queues of the large-set pass, sized for n
// (batch members use the hub's slots).
tim_status ensure_big(tim_ctx* c, int64_t n) {
  if (c->hub) return TIM_OK;
  // slots sized for a larger graph serve a smaller one (stamps are epochs, never cleared between sets)
  if (c->big_slots > 0 && c->big_n >= n) return TIM_OK;
  release(c, c->big_stamp);
  release(c, c->big_queue);
  release(c, c->big_epoch);
  c->big_n = -1;
  // one slot per CU where memory allows (8 bytes per node per slot), up to
  // four while they take at most a sixteenth of it (four blocks per CU share
  // the last tier's sets among them: supercritical graphs give that tier many
  // sets); at most a quarter of the budget, or of the free device memory
  // without one
  const uint64_t per = (uint64_t)n * 8;
  uint64_t room = 0;
  if (c->budget) {
    room = c->budget > c->held ? (c->budget - c->held) / 4 : 0;
  } else {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    room = free_b / 4;
  }
  const int slots = (int)std::max(std::min<uint64_t>((uint64_t)std::max(c->num_cu, 64), room / per),
                                  std::min<uint64_t>((uint64_t)std::max(4 * c->num_cu, 64), room / 4 / per));
  if (slots < 1)
    return fail(TIM_EBUDGET, "budget too small for the large-set pass (needs %llu bytes)",
                (unsigned long long)per * 4);
  TIM_TRY(ensure(c, c->big_stamp, (size_t)slots * (size_t)n * 4, "large-set stamps"));
  TIM_TRY(ensure(c, c->big_queue, (size_t)slots * (size_t)n * 4, "large-set queues"));
  TIM_TRY(ensure(c, c->big_epoch, (size_t)slots * 4, "large-set epochs"));
  HIP_TRY(hipMemsetAsync(c->big_stamp.p, 0, c->big_stamp.bytes, c->stream));
  HIP_TRY(hipMemsetAsync(c->big_epoch.p, 0, c->big_epoch.bytes, c->stream));
  c->big_slots = slots;
  c->big_n = n;
  return TIM_OK;
}

struct Totals {
  uint64_t count = 0, deferred = 0, width = 0, nodes = 0, covered = 0, pool_used = 0;
  u128 kappa = 0;
};

// ---- batches: one sampling launch for the requests of many queries ----
//
// Each query of a batch runs the same host code as tim_run on a context of
// its own, in a thread of its own.  Where that code would launch a sampler,
// it hands its SampleArgs to the hub and waits.  The hub's scheduler thread
// gathers the requests (until every query in flight has one waiting, or a
// short window after the first has passed), lays them out as a job table
// and runs them as one multi-job launch per (model, mode) on its stream,
// then returns each query its counters.  Every set is a function of its own
// keys, so each query's results are those of tim_run alone.

struct Pending {
  int model = 0, mode = 0;
  bool wc = true;
  SampleArgs a;
  hipEvent_t ready = nullptr;  // the query's stream has reached the request
  bool done = false;
  tim_status st = TIM_OK;
  std::string err;
  unsigned long long h[tim::kCtrCount];
};

struct Hub {
  int device = 0, num_cu = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::vector<Pending*> waiting;
  std::chrono::steady_clock::time_point first_wait;
  int alive = 0;  // workers that have not run out of queries
  bool stop = false;
  std::chrono::microseconds window{1000};
  uint64_t limit = 0;         // device memory of the batch
  uint64_t member_budget = 0; // each query's share
  // job table and counters of a round (pinned host mirrors)
  SampleArgs* d_jobs = nullptr;
  SampleArgs* h_jobs = nullptr;
  unsigned long long* d_ctr = nullptr;
  unsigned long long* h_ctr = nullptr;
  size_t cap = 0;
  // last-tier slots shared by every job
  uint32_t* big_stamp = nullptr;
  int32_t* big_queue = nullptr;
  uint32_t* big_epoch = nullptr;
  int big_slots = 0;
  uint64_t big_stride = 0;
  uint64_t big_bytes = 0;
  int grid0[2][3][2] = {};  // tier-0 blocks per CU [model][mode][wc]
  int grid1[3][2] = {};     // IC tier-1 blocks per CU
  int grid_chain[3] = {};   // LT long-chain tier blocks per CU
  uint64_t emit_waves[2] = {0, 0};
  // per-launch timing into the owning context's profile (when it is on)
  tim_ctx* owner = nullptr;
  hipEvent_t pev[3] = {nullptr, nullptr, nullptr};
  // statistics
  uint64_t rounds = 0, jobs = 0, launches = 0, max_jobs = 0;
  uint64_t kpt_steps = 0, kpt_graph_launches = 0;  // the device-driven KptEstimation of tim_run_batch
  // RR pool: device memory granted to NodeSelection by the bytes its theta sets need
  std::mutex mem_mu;
  std::condition_variable mem_cv;
  uint64_t rr_total = 0, rr_free = 0, rr_peak = 0;
  uint64_t next_ticket = 0, serving_ticket = 0;  // grants are served in request order
  uint64_t held = 0;                             // grants that had to wait for memory
  double held_ms = 0.0;
};

// NodeSelection of a batch member (Algorithm 1 over theta sets) is admitted
// by the device memory its collection needs: theta * E|R| * 4 bytes for the
// node pool plus the per-set offsets and the inverted index (resident_bytes,
// from the mean size of the last KptEstimation round).  The grant comes from
// the hub's RR pool, in request order; a request that does not fit waits
// until earlier grants are returned.  One larger than the whole pool gets
// the whole pool and runs its collection in regenerated chunks (A10).  The
// member's budget is its share plus the grant while NodeSelection runs.
void release_transients(tim_ctx* c);
uint64_t transient_bytes(tim_ctx* c);

uint64_t hub_admit(tim_ctx* c, uint64_t need) {
  Hub* h = c->hub;
  const uint64_t grant = std::min(need, h->rr_total);
  const auto t0 = std::chrono::steady_clock::now();
  std::unique_lock<std::mutex> lk(h->mem_mu);
  const uint64_t ticket = h->next_ticket++;
  bool waited = false;
  while (!(h->serving_ticket == ticket && h->rr_free >= grant)) {
    waited = true;
    h->mem_cv.wait(lk);
  }
  h->serving_ticket += 1;
  h->rr_free -= grant;
  h->rr_peak = std::max(h->rr_peak, h->rr_total - h->rr_free);
  if (waited) {
    h->held += 1;
    h->held_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  c->budget = c->share + grant;
  h->mem_cv.notify_all();  // the next ticket may fit too
  return grant;
}

void hub_return(tim_ctx* c, uint64_t grant) {
  Hub* h = c->hub;
  // back within its share; buffers that fit in it stay for the next query (a free waits for the device)
  if (c->held > c->share) release_transients(c);
  c->budget = c->share;
  std::lock_guard<std::mutex> lk(h->mem_mu);
  h->rr_free += grant;
  h->mem_cv.notify_all();
}

// Blocks a request waits in until its round has run.
void hub_submit(Hub* h, Pending* p) {
  std::unique_lock<std::mutex> lk(h->mu);
  if (h->waiting.empty()) h->first_wait = std::chrono::steady_clock::now();
  h->waiting.push_back(p);
  h->cv_sched.notify_one();
  h->cv_done.wait(lk, [&] { return p->done; });
}

// IC launches of fewer sets than this cannot fill the chip with 8-lane
// segments: they last as long as their largest set takes to cross its BFS
// levels, so they run the 64-lane shape instead.  Stored sets take it too,
// with the node-pool bound of that shape (tier0_cap), except in the chunked
// collections, which plan their pool for the context's shape.  Batched
// launches keep theirs.
constexpr uint64_t kWideLaunchSets = 262144;

// Lanes per set of the IC first tier for a launch of `count` sets.
int launch_lanes(const tim_ctx* c, int model, int mode, uint64_t count) {
  if (c->wide_small && !c->hub && model == TIM_MODEL_IC && count < kWideLaunchSets &&
      (mode != tim::kModeEmit || c->emit_wave_sets == 0))
    return 64;
  return c->seg_lanes;
}

// Blocks of the tier-0 sampler over `count` sets (and its wavefronts).
uint64_t sample_grid(const tim_ctx* c, int model, int mode, bool wc, uint64_t count, uint64_t* waves) {
  const int lanes = launch_lanes(c, model, mode, count);
  const int per_cu = model == TIM_MODEL_TRIGGER ? c->grid_trig[mode]
                     : model != TIM_MODEL_IC ? c->grid_lt[mode]
                     : lanes == c->seg_lanes ? c->grid_ic[mode][wc ? 1 : 0]
                                             : c->grid_ic_wide[mode][wc ? 1 : 0];
  const uint64_t waves_per_block = model == TIM_MODEL_LT ? 2 : 4;
  uint64_t sets_per_block = model == TIM_MODEL_IC ? 4 * (64 / (uint64_t)lanes) : model == TIM_MODEL_LT ? 128 : 16;
  if (mode == tim::kModeEmit && c->emit_wave_sets)
    sets_per_block = std::max<uint64_t>(sets_per_block, waves_per_block * c->emit_wave_sets);
  uint64_t grid = (uint64_t)per_cu * (uint64_t)c->num_cu;
  grid = std::min<uint64_t>(grid, (count + sets_per_block - 1) / sets_per_block);
  if (grid < 1) grid = 1;
  if (waves) *waves = grid * waves_per_block;
  return grid;
}

// Wavefronts of the tier-0 launch over `count` sets (the only tier that
// reserves node-pool slices; the others reserve exactly what they store).
uint64_t emit_waves(const tim_ctx* c, int model, uint64_t count) {
  if (c->hub && model != TIM_MODEL_TRIGGER) return c->hub->emit_waves[model];  // any wavefront of a batched launch may visit a job
  uint64_t waves = 0, w2 = 0;
  sample_grid(c, model, tim::kModeEmit, true, count, &waves);
  sample_grid(c, model, tim::kModeEmit, false, count, &w2);
  return std::max(waves, w2);
}

// Largest set tier 0 stores (its LDS queue or chain) in emit launches of
// `count` sets.
uint64_t tier0_cap(const tim_ctx* c, int model, uint64_t count) {
  return tim::tier0_set_cap(model, launch_lanes(c, model, tim::kModeEmit, std::min(count, kMaxLaunchSets)));
}

// Node-pool slice for launches of `count` sets holding about `nodes`
// entries: about a quarter of a wavefront's share, a power of two between
// four times the largest tier-0 set and max(slice_cap, that).
uint32_t pick_slice(const tim_ctx* c, int model, uint64_t count, uint64_t nodes) {
  const uint64_t per_wave = nodes / std::max<uint64_t>(1, emit_waves(c, model, std::min(count, kMaxLaunchSets)));
  const uint32_t lo = (uint32_t)(4 * tier0_cap(c, model, count));
  const uint32_t hi = std::max(lo, c->slice_cap);
  uint32_t s = lo;
  while (s < hi && (uint64_t)s * 8 <= per_wave) s <<= 1;
  return std::min(s, hi);
}

// Node-pool entries that emit launches of `count` sets with `nodes` entries
// need at most with slices of `slice` entries.  A wavefront leaves unused
// less than one set (at most `cap` entries) at a slice boundary, and it
// crosses a boundary once per slice - cap entries stored plus once more
// after its last slice, whose rest (at most a slice) is also lost.
uint64_t pool_need(const tim_ctx* c, int model, uint64_t count, uint64_t nodes, uint32_t slice) {
  const uint64_t cap = tier0_cap(c, model, count);
  const uint64_t launches = (count + kMaxLaunchSets - 1) / kMaxLaunchSets;
  const uint64_t waves = emit_waves(c, model, std::min(count, kMaxLaunchSets));
  const uint64_t boundary = (nodes * cap + (slice - cap) - 1) / (slice - cap);
  return nodes + boundary + launches * waves * ((uint64_t)slice + cap);
}

// One sampling launch pair (wave/lane-level pass, then the large-set pass)
// over sets [first, first+count) with count <= kMaxLaunchSets.  Emit mode
// writes into the node pool from entry pool_base on and records set offsets
// at set_start[set_offset ..].
tim_status sample_launch(tim_ctx* c, const tim_graph* g, int model, int mode, uint64_t seed, uint32_t phase,
                         uint64_t first, uint64_t count, int k, uint64_t* widths, uint32_t* sizes,
                         uint64_t set_offset, uint64_t pool_base, Totals* t) {
  if (model != TIM_MODEL_LT) TIM_TRY(ensure_big(c, g->n));  // the LT long-chain tier needs no slots
  TIM_TRY(ensure(c, c->list1, count * 8, "deferred-set list"));
  if (model != TIM_MODEL_LT) TIM_TRY(ensure(c, c->list2, count * 8, "deferred-set list"));
  SampleArgs a;
  memset(&a, 0, sizeof(a));
  a.g.off = g->off;
  a.g.off32 = g->off32;
  a.g.src = g->src;
  a.g.thr = g->thr;
  a.g.lthr = g->lthr;
  a.g.toff = g->toff;
  a.g.tthr = g->tthr;
  a.g.tset = g->tset;
  a.g.tmem = g->tmem;
  a.g.n = g->n;
  a.g.m = g->m;
  a.seed = seed;
  a.phase = phase;
  a.first = first;
  a.count = count;
  a.k = k;
  a.ctr = c->ctr;
  a.widths = widths;
  a.sizes = sizes;
  if (mode == tim::kModeWidth || (mode == tim::kModeEmit && c->emit_kappa_k > 0)) {
    TIM_TRY(ensure(c, c->wbuf, count * 4, "width buffer"));
    a.wbuf = c->wbuf.as<uint32_t>();
    if (mode == tim::kModeEmit) a.k = c->emit_kappa_k;
  }
  if (mode == tim::kModeEmit) {
    const uint64_t cap = c->pool.bytes / 4;
    a.pool = c->pool.as<int32_t>() + std::min(pool_base, cap);
    a.pool_cap = pool_base < cap ? cap - pool_base : 0;
    a.pool_base = pool_base;
    a.pool_chunk = c->slice;
    a.set_start = c->set_start.as<uint64_t>() + set_offset;
    a.set_len = c->set_len.as<uint32_t>() + set_offset;
  }
  a.seed_bits = c->seed_bits.as<uint32_t>();
  a.list1 = c->list1.as<uint64_t>();
  a.list2 = c->list2.as<uint64_t>();
  a.big_stamp = c->big_stamp.as<uint32_t>();
  a.big_queue = c->big_queue.as<int32_t>();
  a.big_epoch = c->big_epoch.as<uint32_t>();
  a.big_slots = c->big_slots;
  a.big_stride = (uint64_t)c->big_n;
  const bool wc = g->thr == nullptr;
  const unsigned long long* h = c->ctr_host;
  Pending req;
  if (c->hub) {
    // counters and last-tier slots are filled in by the hub
    a.ctr = nullptr;
    req.model = model;
    req.mode = mode;
    req.wc = wc;
    req.a = a;
    HIP_TRY(hipEventRecord(c->ready_ev, c->stream));
    req.ready = c->ready_ev;
    hub_submit(c->hub, &req);
    if (req.st != TIM_OK) return fail(req.st, "%s", req.err.c_str());
    h = req.h;
  } else {
    const uint64_t grid0 = sample_grid(c, model, mode, wc, count, nullptr);
    const uint64_t grid1 = (uint64_t)(model == TIM_MODEL_IC        ? c->grid_ic64[mode][wc ? 1 : 0]
                                      : model == TIM_MODEL_TRIGGER ? c->grid_trig1[mode]
                                                                   : c->grid_lt_chain[mode]) *
                           (uint64_t)c->num_cu;
    tim::launch_clear_counters(c->ctr, c->stream);
    if (c->prof_on) HIP_TRY(hipEventRecord(c->pev[0], c->stream));
    tim::launch_sample(model, mode, a, launch_lanes(c, model, mode, count), (int)grid0, (int)grid1, c->stream,
                       c->prof_on ? c->pev[1] : nullptr);
    if (c->prof_on) HIP_TRY(hipEventRecord(c->pev[2], c->stream));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(c->ctr_host, c->ctr, tim::kCtrCount * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  if (h[tim::kCtrList1] > count || h[tim::kCtrList2] > count) return fail(TIM_EDEVICE, "deferred-set list overflow");
  t->count += count;
  t->deferred += h[tim::kCtrList1];
  for (int tier = 0; tier < 3; ++tier) {
    const unsigned long long* acc = h + tim::kCtrAcc + tim::kAccStride * tier;
    t->kappa += ((u128)acc[tim::kAccKappaHi] << 64) | (u128)acc[tim::kAccKappaLo];
    t->width += acc[tim::kAccWidth];
    t->nodes += acc[tim::kAccNodes];
    t->covered += acc[tim::kAccCovered];
  }
  t->pool_used += h[tim::kCtrPoolCursor];
  if (c->prof_on && !c->hub && model != TIM_MODEL_TRIGGER) {  // the profile covers the IC and LT kernels
    float ms_main = 0.f, ms_big = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms_main, c->pev[0], c->pev[1]));
    HIP_TRY(hipEventElapsedTime(&ms_big, c->pev[1], c->pev[2]));
    // launches in the 64-lane shape are kept apart, so that the sampler[][]
    // entries describe one kernel each
    tim_kernel_profile& p = (model == TIM_MODEL_IC && launch_lanes(c, model, mode, count) != c->seg_lanes)
                                ? c->prof.ic_wide[mode]
                                : c->prof.sampler[model][mode];
    const unsigned long long* acc0 = h + tim::kCtrAcc;
    const uint64_t sets = count - h[tim::kCtrList1];
    const uint64_t nodes = acc0[tim::kAccNodes], edges = acc0[tim::kAccWidth];
    uint64_t bytes;
    if (model == TIM_MODEL_IC) bytes = 16 * nodes + (g->thr ? 8 : 4) * edges;
    else if (model == TIM_MODEL_TRIGGER) bytes = kTriggerNodeBytes * nodes;
    else bytes = 20 * nodes;
    if (mode == tim::kModeEmit) bytes += 4 * nodes + 12 * sets;
    p.launches += 1;
    p.kernel_ms += ms_main;
    p.sets += sets;
    p.nodes += nodes;
    p.edges += edges;
    p.bytes += bytes;
    p.large_launches += 1;
    p.large_ms += ms_big;
    p.deferred += h[tim::kCtrList1];
  }
  return TIM_OK;
}

// Sets per width- or coverage-mode launch: kMaxLaunchSets, or fewer where
// the budget leaves less than four times their deferral lists and widths.
uint64_t launch_cap(const tim_ctx* c) {
  if (!c->budget) return kMaxLaunchSets;
  const uint64_t room = c->budget > c->held ? c->budget - c->held : 0;
  return std::max<uint64_t>(4096, std::min<uint64_t>(kMaxLaunchSets, room / 4 / 20));
}

// Width and coverage passes keep nothing in the node pool or the index, and a
// round kept for RefineKPT is only a shortcut (its flag falls with it).  On a
// budget, the buffers that earlier steps or queries left are released before
// such a pass when they would hold its launches (launch_cap) below 2^20 sets,
// or below `count` if fewer; kept buffers that leave more room stay for reuse.
void room_for_counts(tim_ctx* c, uint64_t count) {
  if (!c->budget) return;
  const uint64_t want = 4 * 20 * std::min<uint64_t>(count, 1ull << 20);
  const uint64_t own = c->list1.bytes + c->list2.bytes + c->wbuf.bytes;
  const uint64_t room = c->budget > c->held ? c->budget - c->held : 0;
  if (room + own < want && transient_bytes(c) > own) release_transients(c);
}

// Width or coverage mode over any number of sets, in launches of bounded size.
tim_status sample_counts(tim_ctx* c, const tim_graph* g, int model, int mode, uint64_t seed, uint32_t phase,
                         uint64_t first, uint64_t count, int k, uint64_t* widths, uint32_t* sizes, Totals* t) {
  room_for_counts(c, count);
  const uint64_t cap = launch_cap(c);
  for (uint64_t done = 0; done < count;) {
    const uint64_t part = std::min(count - done, cap);
    TIM_TRY(sample_launch(c, g, model, mode, seed, phase, first + done, part, k, widths ? widths + done : nullptr,
                          sizes ? sizes + done : nullptr, 0, 0, t));
    done += part;
  }
  return TIM_OK;
}

// Emit mode: sets [first, first+count) into the node pool (set_start /
// set_len per set).  expect_nodes sizes the pool; a short pool is regrown to
// what the exact total guarantees (pool_need) and the sets regenerated.
tim_status emit_sets(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, uint32_t phase, uint64_t first,
                     uint64_t count, uint64_t expect_nodes, uint64_t* widths, Totals* t_out) {
  c->stored.valid = false;
  TIM_TRY(ensure(c, c->set_start, count * 8, "set offsets"));
  TIM_TRY(ensure(c, c->set_len, count * 4, "set sizes"));
  c->slice = pick_slice(c, model, count, expect_nodes);
  TIM_TRY(ensure(c, c->pool, pool_need(c, model, count, std::max<uint64_t>(expect_nodes, 1024), c->slice) * 4,
                 "RR node pool"));
  for (int attempt = 0; attempt < 2; ++attempt) {
    Totals t;
    for (uint64_t done = 0; done < count;) {
      const uint64_t part = std::min(count - done, kMaxLaunchSets);
      TIM_TRY(sample_launch(c, g, model, tim::kModeEmit, seed, phase, first + done, part, 0,
                            widths ? widths + done : nullptr, nullptr, done, t.pool_used, &t));
      done += part;
    }
    if (t.pool_used * 4 <= c->pool.bytes) {
      *t_out = t;
      return TIM_OK;
    }
    TIM_TRY(ensure(c, c->pool, pool_need(c, model, count, t.nodes, c->slice) * 4, "RR node pool"));
  }
  return fail(TIM_EDEVICE, "node pool still short after regrowing");
}

// Emit mode into c->rr_off / c->rr_nodes: a flat CSR of the sets in id order.
tim_status sample_store(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, uint32_t phase, uint64_t first,
                        uint64_t count, uint64_t expect_nodes, uint64_t* widths, Totals* t_out) {
  Totals t;
  TIM_TRY(emit_sets(c, g, model, seed, phase, first, count, expect_nodes, widths, &t));
  TIM_TRY(ensure(c, c->rr_off, (count + 1) * 8, "RR set offsets"));
  TIM_TRY(ensure(c, c->rr_nodes, t.nodes * 4, "RR nodes"));
  TIM_TRY(ensure(c, c->scan_tmp, tim::scan_temp_bytes(std::max<uint64_t>(count, (uint64_t)g->n + 1)), "scan"));
  tim::launch_scan_u32_to_i64(c->set_len.as<uint32_t>(), c->rr_off.as<int64_t>(), count, c->scan_tmp.p, c->stream);
  tim::launch_compact(c->pool.as<int32_t>(), c->set_start.as<uint64_t>(), c->set_len.as<uint32_t>(),
                      c->rr_off.as<int64_t>(), c->rr_nodes.as<int32_t>(), count, c->stream);
  HIP_TRY(hipGetLastError());
  *t_out = t;
  return TIM_OK;
}

// Greedy maximum coverage over a CSR collection in device memory.
// Greedy maximum coverage over a collection in device memory, in CSR layout
// (set_off) or in the node-pool layout of an emit launch (set_start/set_len).
// k = 1 needs only the coverage counts; larger k builds the inverted index.
// TIM_GREEDY_BUCKETS=0 keeps the greedy's counts and index on per-entry device atomics.
bool greedy_buckets() {
  static const bool on = [] {
    const char* e = getenv("TIM_GREEDY_BUCKETS");
    return !(e && e[0] == '0');
  }();
  return on;
}

tim_status greedy(tim_ctx* c, int64_t n, uint64_t nsets, const int64_t* set_off, const uint64_t* set_start,
                  const uint32_t* set_len, const int32_t* nodes, uint64_t total, int k, int32_t* seeds,
                  uint64_t* gains) {
  if (nsets >= 0xFFFFFFFFull) return fail(TIM_EINVAL, "more than 2^32-1 sets in one collection");
  const bool index = k > 1;
  TIM_TRY(ensure(c, c->cnt, (size_t)n * 4, "coverage counts"));
  if (index) {
    TIM_TRY(ensure(c, c->fill, (size_t)n * 4, "index cursors"));
    TIM_TRY(ensure(c, c->inv_off, (size_t)(n + 1) * 8, "index offsets"));
    TIM_TRY(ensure(c, c->inv_sets, total * 4, "index entries"));
    TIM_TRY(ensure(c, c->scan_tmp, tim::scan_temp_bytes((uint64_t)n + 1), "scan"));
  }
  TIM_TRY(ensure(c, c->covered, nsets, "covered marks"));
  TIM_TRY(ensure(c, c->selected, (size_t)n, "selected marks"));
  TIM_TRY(ensure(c, c->best, (size_t)k * 8, "argmax keys"));
  tim::GreedyArgs a;
  memset(&a, 0, sizeof(a));
  a.n = n;
  a.nsets = nsets;
  a.total = total;
  a.set_off = set_off;
  a.set_start = set_start;
  a.set_len = set_len;
  a.nodes = nodes;
  a.cnt = c->cnt.as<uint32_t>();
  if (index) {
    a.fill = c->fill.as<uint32_t>();
    a.inv_off = c->inv_off.as<int64_t>();
    a.inv_sets = c->inv_sets.as<uint32_t>();
    a.scan_temp = c->scan_tmp.p;
  }
  a.covered = c->covered.as<uint8_t>();
  a.selected = c->selected.as<uint8_t>();
  a.best = c->best.as<unsigned long long>();
  // the counting sort by node range where its workspace fits the budget, else per-entry device atomics
  // (under a budget only while it takes at most half of it, so that later allocations of the run keep room)
  const size_t wb = greedy_buckets() ? tim::bucket_workspace_bytes(n, total, index) : 0;
  if (wb && nsets && (!c->budget || c->held - c->bucket.bytes + wb <= c->budget / 2) &&
      ensure(c, c->bucket, wb, "greedy workspace") == TIM_OK)
    a.bkt = c->bucket.p;
  if (c->prof_on) HIP_TRY(hipEventRecord(c->pev[0], c->stream));
  if (index) tim::launch_index(a, c->stream);
  else tim::launch_counts(a, c->stream);
  if (c->prof_on) HIP_TRY(hipEventRecord(c->pev[1], c->stream));
  tim::launch_greedy(a, k, c->stream);
  if (c->prof_on) HIP_TRY(hipEventRecord(c->pev[2], c->stream));
  HIP_TRY(hipGetLastError());
  std::vector<unsigned long long> keys((size_t)k);
  HIP_TRY(hipMemcpyAsync(keys.data(), a.best, (size_t)k * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->prof_on) {
    float ms_index = 0.f, ms_greedy = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms_index, c->pev[0], c->pev[1]));
    HIP_TRY(hipEventElapsedTime(&ms_greedy, c->pev[1], c->pev[2]));
    c->prof.index_calls += 1;
    c->prof.index_ms += ms_index;
    c->prof.greedy_ms += ms_greedy;
  }
  for (int j = 0; j < k; ++j) {
    seeds[j] = (int32_t)(0xFFFFFFFFull - (keys[j] & 0xFFFFFFFFull));
    if (gains) gains[j] = keys[j] >> 32;
  }
  return TIM_OK;
}

// ---- greedy over a phase's sets under the device-memory budget ----
//
// The paper keeps the whole collection R in memory (R, of lambda / KPT+ sets,
// dominates its memory use: Section 7.4).  When the sets and their index do not
// fit, a prefix of the sets is kept with its index and the rest is
// regenerated from its keys in chunks: once to add its memberships to the
// counts, then after every greedy step to take the newly covered sets out of
// them.  Sets are a pure function of (seed, phase, id), so this is the same
// collection and the same greedy, step for step.

float elapsed_ms(tim_ctx* c);

struct CollectionStats {
  uint64_t nodes = 0, width = 0;  // of the collection (each set counted once)
  uint64_t resident = 0;          // sets kept with their index
  uint64_t chunk = 0;             // sets per regenerated chunk (0: none)
  uint64_t regenerated = 0;       // set generations beyond the first
  uint64_t store_bytes = 0;
  float ms_sample = 0.f, ms_greedy = 0.f;
};

DevBuf* const* transient_bufs(tim_ctx* c, size_t* n) {
  static thread_local DevBuf* bufs[18];
  DevBuf* list[] = {&c->list1,  &c->list2,   &c->wbuf,    &c->pool,     &c->set_start, &c->set_len,
                    &c->rr_off, &c->rr_nodes, &c->sizes,  &c->cnt,      &c->fill,      &c->inv_off,
                    &c->inv_sets, &c->covered, &c->selected, &c->best, &c->scan_tmp, &c->bucket};
  for (size_t i = 0; i < 18; ++i) bufs[i] = list[i];
  *n = 18;
  return bufs;
}

uint64_t transient_bytes(tim_ctx* c) {
  size_t nb = 0;
  DevBuf* const* b = transient_bufs(c, &nb);
  uint64_t t = 0;
  for (size_t i = 0; i < nb; ++i) t += b[i]->bytes;
  return t;
}

void release_transients(tim_ctx* c) {
  c->stored.valid = false;
  size_t nb = 0;
  DevBuf* const* b = transient_bufs(c, &nb);
  (void)hipStreamSynchronize(c->stream);
  for (size_t i = 0; i < nb; ++i) release(c, *b[i]);
}

// Bytes a collection may take: the budget (without one, 90% of the free
// device memory) less what the context holds for other purposes.
tim_status collection_room(tim_ctx* c, uint64_t* room) {
  const uint64_t trans = transient_bytes(c);
  const uint64_t other = c->held - trans;
  if (c->budget) {
    *room = c->budget > other ? c->budget - other : 0;
    return TIM_OK;
  }
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  *room = (uint64_t)(0.9 * (double)(free_b + trans));
  return TIM_OK;
}

uint64_t lists_per_set(int model) { return model == TIM_MODEL_IC ? 16 : 8; }

// Peak bytes of the all-resident path for `count` sets of `nodes` entries
// (node pool, per-set starts and sizes, inverted index).
uint64_t resident_bytes(const tim_ctx* c, int64_t n, int model, uint64_t count, uint64_t nodes, int k) {
  const uint64_t lists = std::min(count, kMaxLaunchSets) * lists_per_set(model);
  const uint64_t emit = count * 12 + pool_need(c, model, count, nodes, pick_slice(c, model, count, nodes)) * 4;
  const uint64_t index = (uint64_t)n * 17 + 8 + nodes * 4 + count + 8 * (uint64_t)k +
                         tim::scan_temp_bytes((uint64_t)n + 1) + 17 * 256;
  return lists + emit + index;
}

// Regenerates sets [from, to) of a phase into the node pool, `*chunk` sets at
// a time (halved while a chunk does not fit), and hands every chunk to fn.
template <class F>
tim_status for_chunks(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, uint32_t phase, uint64_t from,
                      uint64_t to, uint64_t* chunk, double nodes_per_set, Totals* tot, F fn) {
  for (uint64_t a = from; a < to;) {
    const uint64_t len = std::min(*chunk, to - a);
    Totals t;
    const tim_status st = emit_sets(c, g, model, seed, phase, a, len, (uint64_t)(nodes_per_set * (double)len) + 1024,
                                    nullptr, &t);
    if (st == TIM_EBUDGET && len > 64) {
      *chunk = len / 2;
      continue;
    }
    TIM_TRY(st);
    fn(a, len);
    HIP_TRY(hipGetLastError());
    if (tot) {
      tot->nodes += t.nodes;
      tot->width += t.width;
    }
    a += len;
  }
  return TIM_OK;
}

// Sets of phase `phase` with ids [0, count): the greedy of Algorithm 1
// on them, keeping as many as the budget allows resident.
// expect_nodes estimates their total size.
tim_status collection_greedy(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, uint32_t phase,
                             uint64_t count, int k, uint64_t expect_nodes, int32_t* seeds, uint64_t* gains,
                             CollectionStats* st) {
  if (count >= 0xFFFFFFFFull) return fail(TIM_EINVAL, "more than 2^32-1 sets in one collection");
  const int64_t n = g->n;
  uint64_t room = 0;
  TIM_TRY(collection_room(c, &room));
  HIP_TRY(hipEventRecord(c->ev[0], c->stream));
  if (count <= c->resident_limit && resident_bytes(c, n, model, count, expect_nodes, k) <= room) {
    // the sets stay in the node pool as the samplers left them (no compaction)
    Totals t;
    tim_status s0 = emit_sets(c, g, model, seed, phase, 0, count, expect_nodes, nullptr, &t);
    if (s0 == TIM_OK) {
      // the estimate was ahead of the sets: their actual size decides whether the index fits too
      expect_nodes = std::max(expect_nodes, t.nodes);
      uint64_t room2 = 0;  // counts the buffers the context already holds as usable
      TIM_TRY(collection_room(c, &room2));
      if (resident_bytes(c, n, model, count, t.nodes, k) <= room2) {
        HIP_TRY(hipEventRecord(c->ev[1], c->stream));
        st->ms_sample = elapsed_ms(c);
        HIP_TRY(hipEventRecord(c->ev[0], c->stream));
        s0 = greedy(c, n, count, nullptr, c->set_start.as<uint64_t>(), c->set_len.as<uint32_t>(),
                    c->pool.as<int32_t>(), t.nodes, k, seeds, gains);
        if (s0 == TIM_OK) {
          HIP_TRY(hipEventRecord(c->ev[1], c->stream));
          st->ms_greedy = elapsed_ms(c);
          st->nodes = t.nodes;
          st->width = t.width;
          st->resident = count;
          st->store_bytes = c->pool.bytes + c->set_start.bytes + c->set_len.bytes +
                            (k > 1 ? c->inv_sets.bytes + c->inv_off.bytes : 0);
          return TIM_OK;
        }
      } else {
        s0 = TIM_EBUDGET;
      }
    }
    // out of device memory on the way: the chunked plan below regenerates instead
    if (s0 != TIM_ENOMEM && s0 != TIM_EBUDGET) return s0;
    HIP_TRY(hipEventRecord(c->ev[0], c->stream));
  }

  // ---- plan: a chunk size for the regenerated part, then the resident prefix
  release_transients(c);
  TIM_TRY(collection_room(c, &room));
  struct SliceScope {
    tim_ctx* c;
    ~SliceScope() {
      c->slice_cap = c->slice_cap_set;
      c->emit_wave_sets = 0;
    }
  } scope{c};
  // small slices, and enough sets per wavefront to fill them: the pool is
  // sized for one chunk
  c->slice_cap = 0;
  c->emit_wave_sets = 64;
  const double nps = count ? std::max(1.0, (double)expect_nodes / (double)count) : 1.0;
  const uint64_t fixed = (uint64_t)n * 5 + count + 8 * (uint64_t)k + 8 * 256;  // cnt, selected, covered, best
  if (fixed >= room)
    return fail(TIM_EBUDGET, "budget too small for the coverage counts of %llu sets (%llu bytes needed, %llu left)",
                (unsigned long long)count, (unsigned long long)fixed, (unsigned long long)room);
  const uint64_t avail = room - fixed;
  // per chunk set: offsets and size, deferral lists, its nodes with their
  // slice-boundary loss, and its share of the last slices of the wavefronts
  const double cap = (double)tier0_cap(c, model, count), slice = 4.0 * cap;
  const double node_bytes = 4.0 * nps * (1.0 + cap / (slice - cap));
  const double slice_per_set = 4.0 * (slice + cap) / (double)c->emit_wave_sets;
  const uint64_t slack_fixed = 4 * (uint64_t)(slice + cap) * 8 + 8 * 256;
  const double per_chunk_set = 12.0 + (double)lists_per_set(model) + node_bytes + slice_per_set;
  uint64_t chunk = avail / 4 > slack_fixed ? (uint64_t)((double)(avail / 4 - slack_fixed) / per_chunk_set) : 0;
  chunk = std::min({chunk, count, kMaxLaunchSets});
  if (chunk < 64 && chunk < count)
    return fail(TIM_EBUDGET, "budget too small to regenerate %llu sets in chunks (%llu bytes left)",
                (unsigned long long)count, (unsigned long long)avail);
  const uint64_t chunk_cost = (uint64_t)((double)chunk * per_chunk_set) + slack_fixed;
  const uint64_t idx_fixed = (uint64_t)n * 12 + 8 + 6 * 256 + tim::scan_temp_bytes(count);  // fill, inv_off, scan
  const double per_res_steady = 8.0 + 8.0 * nps;
  const double per_res_peak = 20.0 + (double)lists_per_set(model) + 4.0 * nps + node_bytes + slice_per_set;
  uint64_t resident = 0;
  if (avail > chunk_cost + idx_fixed) {
    const uint64_t r1 = (uint64_t)((double)(avail - chunk_cost - idx_fixed) / per_res_steady);
    const uint64_t r2 = avail > slack_fixed ? (uint64_t)((double)(avail - slack_fixed) / per_res_peak) : 0;
    resident = std::min({r1, r2, count - 1, c->resident_limit});
  }

  tim::GreedyArgs a;
  memset(&a, 0, sizeof(a));
  a.n = n;
  a.scan_temp = nullptr;
  Totals first_pass;
  if (resident > 0) {
    Totals t;
    tim_status s1 = sample_store(c, g, model, seed, phase, 0, resident, (uint64_t)(nps * (double)resident) + 1024,
                                 nullptr, &t);
    if (s1 == TIM_OK) {
      release(c, c->pool);
      release(c, c->set_start);
      release(c, c->set_len);
      release(c, c->list1);
      release(c, c->list2);
      s1 = ensure(c, c->inv_sets, t.nodes * 4, "index entries");
    }
    if (s1 == TIM_OK) s1 = ensure(c, c->fill, (size_t)n * 4, "index cursors");
    if (s1 == TIM_OK) s1 = ensure(c, c->inv_off, (size_t)(n + 1) * 8, "index offsets");
    if (s1 == TIM_OK) s1 = ensure(c, c->cnt, (size_t)n * 4, "coverage counts");
    if (s1 == TIM_OK) s1 = ensure(c, c->scan_tmp, tim::scan_temp_bytes((uint64_t)n + 1), "scan");
    if (s1 == TIM_EBUDGET) {
      // the prefix came out larger than estimated: regenerate everything instead
      release_transients(c);
      resident = 0;
    } else {
      TIM_TRY(s1);
      a.nsets = resident;
      a.total = t.nodes;
      a.set_off = c->rr_off.as<int64_t>();
      a.nodes = c->rr_nodes.as<int32_t>();
      a.cnt = c->cnt.as<uint32_t>();
      a.fill = c->fill.as<uint32_t>();
      a.inv_off = c->inv_off.as<int64_t>();
      a.inv_sets = c->inv_sets.as<uint32_t>();
      a.scan_temp = c->scan_tmp.p;
      tim::launch_index(a, c->stream);
      HIP_TRY(hipGetLastError());
      first_pass = t;
    }
  }
  TIM_TRY(ensure(c, c->cnt, (size_t)n * 4, "coverage counts"));
  TIM_TRY(ensure(c, c->covered, count, "covered marks"));
  TIM_TRY(ensure(c, c->selected, (size_t)n, "selected marks"));
  TIM_TRY(ensure(c, c->best, (size_t)k * 8, "argmax keys"));
  a.cnt = c->cnt.as<uint32_t>();
  a.covered = c->covered.as<uint8_t>();
  a.selected = c->selected.as<uint8_t>();
  a.best = c->best.as<unsigned long long>();
  if (resident == 0) {
    a.nsets = 0;
    tim::launch_zero_counts(a.cnt, n, c->stream);
  }
  tim::launch_greedy_init(a, count, k, c->stream);

  // memberships of the regenerated part
  TIM_TRY(for_chunks(c, g, model, seed, phase, resident, count, &chunk, nps, &first_pass,
                     [&](uint64_t, uint64_t len) {
                       tim::launch_pool_hist(c->pool.as<int32_t>(), c->set_start.as<uint64_t>(),
                                             c->set_len.as<uint32_t>(), len, a.cnt, c->stream);
                     }));
  HIP_TRY(hipEventRecord(c->ev[1], c->stream));
  st->ms_sample = elapsed_ms(c);
  HIP_TRY(hipEventRecord(c->ev[0], c->stream));
  for (int j = 0; j < k; ++j) {
    tim::launch_argmax_step(a, j, c->stream);
    if (j + 1 == k) break;  // the last choice changes no later step
    tim::launch_cover_step(a, j, c->stream);
    TIM_TRY(for_chunks(c, g, model, seed, phase, resident, count, &chunk, nps, nullptr,
                       [&](uint64_t first, uint64_t len) {
                         tim::launch_pool_cover(a.best + j, c->pool.as<int32_t>(), c->set_start.as<uint64_t>(),
                                                c->set_len.as<uint32_t>(), len, a.covered + first, a.cnt,
                                                c->stream);
                       }));
    st->regenerated += count - resident;
  }
  HIP_TRY(hipGetLastError());
  std::vector<unsigned long long> keys((size_t)k);
  HIP_TRY(hipMemcpyAsync(keys.data(), a.best, (size_t)k * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipEventRecord(c->ev[1], c->stream));
  st->ms_greedy = elapsed_ms(c);
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int j = 0; j < k; ++j) {
    seeds[j] = (int32_t)(0xFFFFFFFFull - (keys[j] & 0xFFFFFFFFull));
    if (gains) gains[j] = keys[j] >> 32;
  }
  st->nodes = first_pass.nodes;
  st->width = first_pass.width;
  st->resident = resident;
  st->chunk = chunk;
  st->store_bytes = transient_bytes(c);
  return TIM_OK;
}

// ---- scalar formulas (binary64, fixed evaluation order) ----
double ln_binom(int64_t n, int k) {
  double s = 0.0;
  for (int i = 0; i < k; ++i) s = s + (std::log((double)(n - i)) - std::log((double)(i + 1)));
  return s;
}

double lambda_eq4(int64_t n, int k, double eps, double ell) {
  const double nd = (double)n;
  return ((8.0 + 2.0 * eps) * nd * ((ell * std::log(nd) + ln_binom(n, k)) + std::log(2.0))) / (eps * eps);
}

int rounds_of(int64_t n) {
  int bits = 0;
  for (uint64_t x = (uint64_t)n; x; x >>= 1) ++bits;
  return bits - 2;
}

uint64_t round_size(int64_t n, double ell, int i) {
  const double nd = (double)n;
  const double a = 6.0 * ell * std::log(nd) + 6.0 * std::log(std::log2(nd));
  return (uint64_t)std::ceil(std::ldexp(a, i));
}

tim_status check_phase_args(const tim_ctx* c, const tim_graph* g, int model, int k) {
  if (!c) return fail(TIM_EINVAL, "null context");
  if (!check_graph(c, g)) return fail(TIM_EINVAL, "graph does not belong to this context");
  if (model != TIM_MODEL_IC && model != TIM_MODEL_LT && model != TIM_MODEL_TRIGGER)
    return fail(TIM_EINVAL, "unknown model %d", model);
  if (model == TIM_MODEL_TRIGGER && !g->toff)
    return fail(TIM_EINVAL, "the graph has no triggering distribution (tim_graph_set_triggering)");
  if (model == TIM_MODEL_TRIGGER && c->hub)
    return fail(TIM_EINVAL, "the general triggering model runs through tim_run, not in batches or servers");
  if (k < 1 || (int64_t)k > g->n) return fail(TIM_EINVAL, "k=%d outside [1, n=%lld]", k, (long long)g->n);
  return TIM_OK;
}

tim_status upload_seed_bits(tim_ctx* c, int64_t n, const int32_t* seeds, int nseeds) {
  const size_t words = (size_t)(n + 31) / 32;
  std::vector<uint32_t> bits(words, 0u);
  for (int j = 0; j < nseeds; ++j) {
    if (seeds[j] < 0 || seeds[j] >= n) return fail(TIM_EINVAL, "seed %d outside [0, n)", seeds[j]);
    bits[(uint32_t)seeds[j] >> 5] |= 1u << ((uint32_t)seeds[j] & 31u);
  }
  TIM_TRY(ensure(c, c->seed_bits, words * 4, "seed bitmap"));
  HIP_TRY(hipMemcpyAsync(c->seed_bits.p, bits.data(), words * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return TIM_OK;
}

float elapsed_ms(tim_ctx* c) {
  float ms = 0.f;
  (void)hipEventSynchronize(c->ev[1]);
  (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
  return ms;
}

// Early KptEstimation rounds whose sets together number at most kGroupSets
// run as the jobs of one multi-job launch (kpt_estimate_impl); a later round
// not predicted to be the last runs paired with the next one while the two
// number at most kPairSets (IC) or kPairSetsLt (LT).  Larger IC pairs lose
// to the single-launch kernel's higher occupancy; LT chains gain up to 2^23.
constexpr uint64_t kGroupSets = 1ull << 19;
constexpr uint64_t kPairSets = 1ull << 21;
constexpr uint64_t kPairSetsLt = 1ull << 23;

// Width-mode sets of rounds i0..i1 of KptEstimation, one job per round
// (phase i, sets [0, c_i)), in one multi-job launch; t[r] receives the totals
// of round i0 + r.  A launch of few sets lasts about as long as its largest
// set takes to cross its BFS levels or chain, so the early rounds, launched
// one by one, each pay that latency; launched together they pay it once.
// Every set is a function of its own keys, so each round's totals are those
// of a launch of that round alone.
tim_status sample_rounds(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, int k, double ell, int i0, int i1,
                         Totals* t) {
  const int J = i1 - i0 + 1;
  if (J < 1 || J > tim::kMaxBatchJobs) return fail(TIM_EINVAL, "%d rounds in one launch", J);
  std::vector<uint64_t> base((size_t)J), cnt((size_t)J);
  uint64_t total = 0, maxc = 0;
  for (int r = 0; r < J; ++r) {
    cnt[(size_t)r] = round_size(g->n, ell, i0 + r);
    base[(size_t)r] = total;
    total += cnt[(size_t)r];
    maxc = std::max(maxc, cnt[(size_t)r]);
  }
  room_for_counts(c, total);
  if (model == TIM_MODEL_IC) TIM_TRY(ensure_big(c, g->n));
  TIM_TRY(ensure(c, c->list1, total * 8, "deferred-set list"));
  if (model == TIM_MODEL_IC) TIM_TRY(ensure(c, c->list2, total * 8, "deferred-set list"));
  TIM_TRY(ensure(c, c->wbuf, total * 4, "width buffer"));
  const size_t table = ((size_t)J * sizeof(SampleArgs) + 255) & ~(size_t)255;
  const size_t ctr_words = (size_t)J * tim::kCtrCount;
  TIM_TRY(ensure(c, c->jobs, table + ctr_words * sizeof(unsigned long long), "job table"));
  unsigned long long* d_ctr = reinterpret_cast<unsigned long long*>(static_cast<char*>(c->jobs.p) + table);
  std::vector<SampleArgs> jobs((size_t)J);
  for (int r = 0; r < J; ++r) {
    SampleArgs& a = jobs[(size_t)r];
    memset(&a, 0, sizeof(a));
    a.g.off = g->off;
    a.g.off32 = g->off32;
    a.g.src = g->src;
    a.g.thr = g->thr;
    a.g.lthr = g->lthr;
    a.g.n = g->n;
    a.g.m = g->m;
    a.seed = seed;
    a.phase = (uint32_t)(i0 + r);
    a.first = 0;
    a.count = cnt[(size_t)r];
    a.k = k;
    a.ctr = d_ctr + (size_t)r * tim::kCtrCount;
    a.wbuf = c->wbuf.as<uint32_t>() + base[(size_t)r];
    a.seed_bits = c->seed_bits.as<uint32_t>();
    a.list1 = c->list1.as<uint64_t>() + base[(size_t)r];
    a.list2 = model == TIM_MODEL_IC ? c->list2.as<uint64_t>() + base[(size_t)r] : nullptr;
    a.big_stamp = c->big_stamp.as<uint32_t>();
    a.big_queue = c->big_queue.as<int32_t>();
    a.big_epoch = c->big_epoch.as<uint32_t>();
    a.big_slots = c->big_slots;
    a.big_stride = (uint64_t)c->big_n;
  }
  const bool wc = g->thr == nullptr;
  const tim::JobTable tab{c->jobs.as<SampleArgs>(), J, 1};
  HIP_TRY(hipMemcpyAsync(c->jobs.p, jobs.data(), (size_t)J * sizeof(SampleArgs), hipMemcpyHostToDevice, c->stream));
  tim::launch_clear_counters_batch(tab, c->stream);
  const uint64_t per_block = model == TIM_MODEL_IC ? 32 : 128;  // sets a tier-0 block holds at once
  const uint64_t full = (uint64_t)c->grid_rounds[model][wc ? 1 : 0] * (uint64_t)c->num_cu;
  const uint64_t grid0 = std::max<uint64_t>(1, std::min(full, (total + per_block - 1) / per_block));
  const uint64_t grid1 =
      (uint64_t)(model == TIM_MODEL_IC ? c->grid_batch1[wc ? 1 : 0] : c->grid_batch_chain) * (uint64_t)c->num_cu;
  if (c->prof_on) HIP_TRY(hipEventRecord(c->pev[0], c->stream));
  tim::launch_sample_batch(model, tim::kModeWidth, wc, tab, (int)grid0, (int)grid1, c->big_slots, maxc, c->stream,
                           c->prof_on ? c->pev[1] : nullptr);
  if (c->prof_on) HIP_TRY(hipEventRecord(c->pev[2], c->stream));
  HIP_TRY(hipGetLastError());
  std::vector<unsigned long long> h(ctr_words);
  HIP_TRY(hipMemcpyAsync(h.data(), d_ctr, ctr_words * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  uint64_t sets = 0, nodes = 0, edges = 0, deferred = 0;
  for (int r = 0; r < J; ++r) {
    const unsigned long long* hr = h.data() + (size_t)r * tim::kCtrCount;
    if (hr[tim::kCtrList1] > cnt[(size_t)r] || hr[tim::kCtrList2] > cnt[(size_t)r])
      return fail(TIM_EDEVICE, "deferred-set list overflow");
    Totals& tr = t[r];
    tr = Totals();
    tr.count = cnt[(size_t)r];
    tr.deferred = hr[tim::kCtrList1];
    for (int tier = 0; tier < 3; ++tier) {
      const unsigned long long* acc = hr + tim::kCtrAcc + tim::kAccStride * tier;
      tr.kappa += ((u128)acc[tim::kAccKappaHi] << 64) | (u128)acc[tim::kAccKappaLo];
      tr.width += acc[tim::kAccWidth];
      tr.nodes += acc[tim::kAccNodes];
      tr.covered += acc[tim::kAccCovered];
    }
    sets += cnt[(size_t)r] - hr[tim::kCtrList1];
    nodes += hr[tim::kCtrAcc + tim::kAccNodes];
    edges += hr[tim::kCtrAcc + tim::kAccWidth];
    deferred += hr[tim::kCtrList1];
  }
  if (c->prof_on) {
    float ms_main = 0.f, ms_big = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms_main, c->pev[0], c->pev[1]));
    HIP_TRY(hipEventElapsedTime(&ms_big, c->pev[1], c->pev[2]));
    tim_kernel_profile& p = c->prof.grouped[model];
    p.launches += 1;
    p.kernel_ms += ms_main;
    p.sets += sets;
    p.nodes += nodes;
    p.edges += edges;
    p.bytes += model == TIM_MODEL_IC ? 16 * nodes + (g->thr ? 8 : 4) * edges : 20 * nodes;
    p.large_launches += 1;
    p.large_ms += ms_big;
    p.deferred += deferred;
  }
  return TIM_OK;
}

// Algorithm 2.  With keep_last, a round that the previous one predicts to be
// the last (its mean kappa already above 0.8 * 2^-i) is stored in the node
// pool while its widths are summed, so that RefineKPT can take its sets
// without generating them again.  Outside batches, the early rounds run
// together (sample_rounds) and are then taken in order exactly as if run one
// by one: the first that stops ends the estimation, the rest are dropped, and
// a round predicted to be the last is run again on its own to be stored.
tim_status kpt_estimate_impl(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, int k, double ell,
                             bool keep_last, tim_kpt_result* out, uint64_t* sets, uint64_t* width) {
  memset(out, 0, sizeof(*out));
  const int imax = rounds_of(g->n);
  out->i_max = imax;
  out->i_last = imax;
  out->c_last = imax >= 1 ? round_size(g->n, ell, imax) : 0;
  room_for_counts(c, out->c_last);  // room for the largest round's launches
  out->kpt_star = 1.0;
  u128 prev_sum = 0;
  uint64_t prev_c = 0, prev_nodes = 0;
  // predicted last: S_{i-1} * 2^i > 0.8 * c_{i-1} * 2^53, evaluated as 5 * S * 2^i > 4 * c * 2^53
  auto predict = [&](int i, uint64_t ci) {
    return keep_last && prev_c > 0 && ci <= kMaxLaunchSets && ((prev_sum * 5) << i) > (((u128)prev_c * 4) << 53);
  };
  // records round i; true when it stops the estimation
  auto finish = [&](int i, uint64_t ci, const Totals& t, bool stored) {
    out->round_c[i] = ci;
    out->round_sum_lo[i] = (uint64_t)t.kappa;
    out->round_sum_hi[i] = (uint64_t)(t.kappa >> 64);
    out->round_width[i] = t.width;
    out->round_nodes[i] = t.nodes;
    if (sets) *sets += ci;
    if (width) *width += t.width;
    prev_sum = t.kappa;
    prev_c = ci;
    prev_nodes = t.nodes;
    // sum/c_i > 2^-i with sum = S * 2^-53 exactly: S * 2^i > c_i * 2^53
    if ((t.kappa << i) <= ((u128)ci << 53)) return false;
    const double sum = std::ldexp((double)t.kappa, -53);
    out->kpt_star = (sum * (double)g->n) / (2.0 * (double)ci);
    out->i_last = i;
    out->c_last = ci;
    if (stored) {
      c->stored.valid = true;
      c->stored.graph = g;
      c->stored.model = model;
      c->stored.seed = seed;
      c->stored.phase = (uint32_t)i;
      c->stored.count = ci;
      c->stored.nodes = t.nodes;
      c->stored.width = t.width;
    }
    return true;
  };
  for (int i = 1; i <= imax;) {
    const uint64_t ci = round_size(g->n, ell, i);
    Totals t;
    const bool predicted = predict(i, ci);
    if (!c->hub && !predicted && model != TIM_MODEL_TRIGGER) {
      // the rounds of few sets run together (up to kGroupSets sets), a later
      // round with the next one (up to kPairSets); under a budget, the
      // group's lists (20 bytes per set) take at most an eighth of the room
      // and are released afterwards, so that what later rounds and the node
      // pool find is what one round per launch leaves
      const uint64_t pair_cap = model == TIM_MODEL_LT ? kPairSetsLt : kPairSets;
      uint64_t group_cap = std::max(kGroupSets, std::min(3 * ci, pair_cap));
      if (c->budget) group_cap = std::min(group_cap, launch_cap(c) / 2);
      int j = i;
      uint64_t tot = ci;
      while (j < imax && j - i + 1 < tim::kMaxBatchJobs) {
        const uint64_t next = round_size(g->n, ell, j + 1);
        if (tot + next > group_cap) break;
        tot += next;
        ++j;
      }
      if (j > i) {
        std::vector<Totals> ts((size_t)(j - i + 1));
        TIM_TRY(sample_rounds(c, g, model, seed, k, ell, i, j, ts.data()));
        if (c->budget)
          for (DevBuf* b : {&c->list1, &c->list2, &c->wbuf, &c->jobs}) release(c, *b);
        int r = i;
        for (; r <= j; ++r) {
          const uint64_t cr = round_size(g->n, ell, r);
          if (r > i && predict(r, cr)) break;  // to be stored: run on its own
          if (finish(r, cr, ts[(size_t)(r - i)], false)) return TIM_OK;
        }
        i = r;
        continue;
      }
    }
    bool stored = false, counted = false;  // counted: the emit summed the round's widths and kappa
    if (predicted) {
      const uint64_t expect = (uint64_t)((double)prev_nodes / (double)prev_c * 1.25 * (double)ci) + 4096;
      uint64_t room = 0;
      TIM_TRY(collection_room(c, &room));
      if (resident_bytes(c, g->n, model, ci, expect, k) + ci * 4 <= room) {
        struct KappaScope {
          tim_ctx* c;
          ~KappaScope() { c->emit_kappa_k = 0; }
        } scope{c};
        c->emit_kappa_k = k;
        const tim_status es = emit_sets(c, g, model, seed, (uint32_t)i, 0, ci, expect, nullptr, &t);
        if (es == TIM_OK) {
          // the sets may have come out larger than estimated: their actual size decides whether
          // RefineKPT's index fits beside them (if not, RefineKPT generates R' again)
          uint64_t room2 = 0;
          TIM_TRY(collection_room(c, &room2));
          stored = resident_bytes(c, g->n, model, ci, t.nodes, k) <= room2;
          counted = true;
          if (!stored) release_transients(c);
        } else if (es == TIM_EBUDGET) {
          // the round's sets came out larger than estimated: sum its widths instead (RefineKPT
          // generates R' again from its keys, with the same sets)
          release_transients(c);
          t = Totals();
        } else {
          return es;
        }
      }
    }
    if (!counted)
      TIM_TRY(sample_counts(c, g, model, tim::kModeWidth, seed, (uint32_t)i, 0, ci, k, nullptr, nullptr, &t));
    if (finish(i, ci, t, stored)) break;
    ++i;
  }
  return TIM_OK;
}

tim_status refine_impl(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, int k, double eps, double ell,
                       double kpt_star, int i_last, uint64_t c_last, uint64_t expect_nodes, int32_t* s_prime,
                       tim_refine_result* out, uint64_t* sets, uint64_t* width) {
  memset(out, 0, sizeof(*out));
  // S'_k: greedy on the sets of the last round of Algorithm 2 - still in
  // the node pool when KptEstimation kept them, else generated again
  CollectionStats cs;
  const tim_ctx::Stored& kept = c->stored;
  bool done = false;
  if (c_last > 0 && kept.valid && kept.graph == g && kept.model == model && kept.seed == seed &&
      kept.phase == (uint32_t)i_last && kept.count == c_last) {
    const tim_status gs = greedy(c, g->n, c_last, nullptr, c->set_start.as<uint64_t>(), c->set_len.as<uint32_t>(),
                                 c->pool.as<int32_t>(), kept.nodes, k, s_prime, nullptr);
    if (gs != TIM_OK && gs != TIM_EBUDGET && gs != TIM_ENOMEM) return gs;
    done = gs == TIM_OK;
    // no room for the index beside the kept sets: R' again from its keys (the same sets), fitted to the budget
    if (!done) release_transients(c);
  }
  if (!done && c_last > 0) {
    TIM_TRY(collection_greedy(c, g, model, seed, (uint32_t)i_last, c_last, k, expect_nodes, s_prime, nullptr, &cs));
    if (sets) *sets += c_last;
    if (width) *width += cs.width;
  } else if (c_last == 0) {
    for (int j = 0; j < k; ++j) s_prime[j] = j;
  }
  c->stored.valid = false;
  // eps', lambda', theta': fresh sets and the fraction that meets S'_k
  const double nd = (double)g->n;
  const double eps_p = 5.0 * std::cbrt(ell * eps * eps / ((double)k + ell));
  const double lambda_p = ((2.0 + eps_p) * ell * nd * std::log(nd)) / (eps_p * eps_p);
  const uint64_t theta_p = (uint64_t)std::ceil(lambda_p / kpt_star);
  TIM_TRY(upload_seed_bits(c, g->n, s_prime, k));
  Totals tc;
  TIM_TRY(sample_counts(c, g, model, tim::kModeCover, seed, TIM_PHASE_REFINE, 0, theta_p, 0, nullptr, nullptr, &tc));
  if (sets) *sets += theta_p;
  // KPT' from that fraction, and KPT+
  const double f = (double)tc.covered / (double)theta_p;
  const double kpt_p = f * nd / (1.0 + eps_p);
  out->eps_prime = eps_p;
  out->lambda_prime = lambda_p;
  out->theta_prime = theta_p;
  out->covered_prime = tc.covered;
  out->kpt_prime = kpt_p;
  out->kpt_plus = kpt_p > kpt_star ? kpt_p : kpt_star;
  return TIM_OK;
}

struct SelectTimes {
  float sample = 0.f, index_greedy = 0.f;
};

tim_status node_select_impl(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, int k, uint64_t theta,
                            uint64_t expect_nodes, int32_t* seeds, uint64_t* gains, tim_select_result* out,
                            SelectTimes* times) {
  std::vector<uint64_t> g_local((size_t)k);
  uint64_t* gp = gains ? gains : g_local.data();
  CollectionStats cs;
  TIM_TRY(collection_greedy(c, g, model, seed, TIM_PHASE_SELECT, theta, k, expect_nodes, seeds, gp, &cs));
  if (times) {
    times->sample = cs.ms_sample;
    times->index_greedy = cs.ms_greedy;
  }
  if (out) {
    memset(out, 0, sizeof(*out));
    out->theta = theta;
    out->nodes = cs.nodes;
    out->width = cs.width;
    uint64_t cov = 0;
    for (int j = 0; j < k; ++j) cov += gp[j];
    out->covered = cov;
    out->store_bytes = cs.store_bytes;
    out->resident_sets = cs.resident;
    out->chunk_sets = cs.chunk;
    out->regenerated_sets = cs.regenerated;
  }
  return TIM_OK;
}

double ell_of(const tim_graph* g, double ell, uint32_t flags) {
  if (!(flags & TIM_FLAG_ELL_ADJUST)) return ell;
  return ell * (1.0 + std::log((flags & TIM_FLAG_PLAIN) ? 2.0 : 3.0) / std::log((double)g->n));
}

// KPT* from the totals of the rounds of a finished KptEstimation (as kpt_estimate_impl computes it).
void kpt_finish_result(const tim_graph* g, tim_kpt_result* out) {
  out->kpt_star = 1.0;
  const int i = out->i_last;
  if (i < 1) return;
  const u128 sum = ((u128)out->round_sum_hi[i] << 64) | (u128)out->round_sum_lo[i];
  const uint64_t ci = out->round_c[i];
  if ((sum << i) <= ((u128)ci << 53)) return;
  out->kpt_star = (std::ldexp((double)sum, -53) * (double)g->n) / (2.0 * (double)ci);
}

// TIM / TIM+; kpt_in (nullable): a KptEstimation already done for this query
// (the batch runs Algorithm 2 for all its queries on the device first).
tim_status run_impl(tim_ctx* c, const tim_graph* g, int model, int k, double eps, double ell, uint64_t seed,
                    uint32_t flags, int32_t* seeds, uint64_t* gains, tim_report* rep,
                    const tim_kpt_result* kpt_in = nullptr) {
  tim_report local;
  tim_report* r = rep ? rep : &local;
  memset(r, 0, sizeof(*r));
  const bool plain = (flags & TIM_FLAG_PLAIN) != 0;
  const double ell_used = ell_of(g, ell, flags);
  r->ell_used = ell_used;
  hipEvent_t t0, t1;
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  auto lap = [&](double* slot) {
    (void)hipEventRecord(t1, c->stream);
    (void)hipEventSynchronize(t1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    *slot = ms;
    (void)hipEventRecord(t0, c->stream);
  };
  (void)hipEventRecord(t0, c->stream);
  tim_status st = TIM_OK;
  if (kpt_in) {
    r->kpt = *kpt_in;
    for (int i = 1; i <= r->kpt.i_last; ++i) {
      r->sets_total += r->kpt.round_c[i];
      r->width_total += r->kpt.round_width[i];
    }
  } else {
    st = kpt_estimate_impl(c, g, model, seed, k, ell_used, !plain, &r->kpt, &r->sets_total, &r->width_total);
  }
  if (st == TIM_OK) lap(&r->ms_kpt);
  // mean set size of the stopping round sizes the node pools
  const int il = r->kpt.i_last;
  const double mean_nodes =
      (il >= 1 && r->kpt.round_c[il]) ? (double)r->kpt.round_nodes[il] / (double)r->kpt.round_c[il] : 16.0;
  double lb = r->kpt.kpt_star;
  std::vector<int32_t> sp((size_t)k);
  if (st == TIM_OK && !plain) {
    st = refine_impl(c, g, model, seed, k, eps, ell_used, r->kpt.kpt_star, r->kpt.i_last, r->kpt.c_last,
                     (uint64_t)(mean_nodes * 1.25 * (double)r->kpt.c_last) + 4096, sp.data(), &r->refine,
                     &r->sets_total, &r->width_total);
    if (st == TIM_OK) {
      lap(&r->ms_refine);
      lb = r->refine.kpt_plus;
      for (int j = 0; j < k && j < 128; ++j) r->s_prime[j] = sp[(size_t)j];
    }
  }
  if (st == TIM_OK) {
    r->lambda = lambda_eq4(g->n, k, eps, ell_used);
    const uint64_t theta = (uint64_t)std::ceil(r->lambda / lb);
    const uint64_t expect = (uint64_t)(mean_nodes * 1.25 * (double)theta) + 4096;
    SelectTimes times;
    uint64_t grant = 0;
    if (c->hub) grant = hub_admit(c, resident_bytes(c, g->n, model, theta, expect, k) + theta * 8);
    st = node_select_impl(c, g, model, seed, k, theta, expect, seeds, gains, &r->select, &times);
    if (c->hub) hub_return(c, grant);
    if (st == TIM_OK) {
      r->ms_select_sample = times.sample;
      r->ms_select_index = 0.0;
      r->ms_select_greedy = times.index_greedy;
      r->sets_total += theta;
      r->width_total += r->select.width;
      r->ms_total = r->ms_kpt + r->ms_refine + r->ms_select_sample + r->ms_select_greedy;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  return st;
}

// Out-edge lists of g (counting sort of its in-edges by source), kept with the
// graph: 8(n+1) + 8m bytes.
tim_status ensure_out_csr(tim_ctx* c, tim_graph* g) {
  if (g->out_off) return TIM_OK;
  const int64_t n = g->n, m = g->m;
  int64_t* off = nullptr;
  int32_t* dst = nullptr;
  uint32_t* eid = nullptr;
  if (hipMalloc(&off, (size_t)(n + 1) * 8) != hipSuccess || hipMalloc(&dst, (size_t)m * 4) != hipSuccess ||
      hipMalloc(&eid, (size_t)m * 4) != hipSuccess) {
    if (off) (void)hipFree(off);
    if (dst) (void)hipFree(dst);
    return fail(TIM_ENOMEM, "out-edge lists: hipMalloc failed");
  }
  tim_status st = ensure(c, c->cnt, (size_t)n * 4, "out-degree counts");
  if (st == TIM_OK) st = ensure(c, c->fill, (size_t)n * 4, "out-list cursors");
  if (st == TIM_OK) st = ensure(c, c->scan_tmp, tim::scan_temp_bytes((uint64_t)n + 1), "scan");
  if (st != TIM_OK) {
    (void)hipFree(off);
    (void)hipFree(dst);
    (void)hipFree(eid);
    return st;
  }
  tim::launch_zero_counts(c->cnt.as<uint32_t>(), n, c->stream);
  tim::launch_zero_counts(c->fill.as<uint32_t>(), n, c->stream);
  tim::launch_out_csr_count(g->src, m, c->cnt.as<uint32_t>(), c->stream);
  tim::launch_scan_u32_to_i64(c->cnt.as<uint32_t>(), off, (uint64_t)n, c->scan_tmp.p, c->stream);
  tim::launch_out_csr_scatter(g->off, g->src, n, m, off, c->fill.as<uint32_t>(), dst, eid, c->stream);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipFree(off);
    (void)hipFree(dst);
    (void)hipFree(eid);
    return fail(TIM_EDEVICE, "building the out-edge lists failed");
  }
  g->out_off = off;
  g->out_dst = dst;
  g->out_eid = eid;
  return TIM_OK;
}

void set_seg_lanes(tim_ctx* c, int lanes) {
  c->seg_lanes = lanes;
  for (int mode = 0; mode < 3; ++mode)
    for (int wc = 0; wc < 2; ++wc) c->grid_ic[mode][wc] = tim::ic_blocks_per_cu(mode, wc != 0, lanes);
}

tim_status check_run_args(const tim_ctx* c, const tim_graph* g, int model, int k, double eps, double ell,
                          const int32_t* seeds) {
  TIM_TRY(check_phase_args(c, g, model, k));
  if (!seeds) return fail(TIM_EINVAL, "seeds is null");
  if (!(eps > 0.0 && eps <= 1.0)) return fail(TIM_EINVAL, "eps must be in (0, 1]");
  if (!(ell >= 0.5)) return fail(TIM_EINVAL, "ell must be >= 0.5");
  return TIM_OK;
}

// ---- batch rounds ----

// One round: the requests in `subs` as one job table, one multi-job launch
// per run of at most kMaxBatchJobs requests of the same (model, mode,
// thresholds), all on the hub's stream.
tim_status hub_round(Hub* h, std::vector<Pending*>& subs) {
  auto cls = [](const Pending* p) { return (p->model * 3 + p->mode) * 2 + (p->wc ? 1 : 0); };
  std::stable_sort(subs.begin(), subs.end(), [&](const Pending* x, const Pending* y) { return cls(x) < cls(y); });
  const size_t J = subs.size();
  if (J > h->cap) {
    (void)hipStreamSynchronize(h->stream);
    if (h->d_jobs) (void)hipFree(h->d_jobs);
    if (h->h_jobs) (void)hipHostFree(h->h_jobs);
    if (h->d_ctr) (void)hipFree(h->d_ctr);
    if (h->h_ctr) (void)hipHostFree(h->h_ctr);
    h->d_jobs = h->h_jobs = nullptr;
    h->d_ctr = h->h_ctr = nullptr;
    h->cap = 0;
    const size_t cap = std::max<size_t>(J, 64);
    HIP_TRY(hipMalloc(&h->d_jobs, cap * sizeof(SampleArgs)));
    HIP_TRY(hipHostMalloc(&h->h_jobs, cap * sizeof(SampleArgs), hipHostMallocDefault));
    HIP_TRY(hipMalloc(&h->d_ctr, cap * tim::kCtrCount * sizeof(unsigned long long)));
    HIP_TRY(hipHostMalloc(&h->h_ctr, cap * tim::kCtrCount * sizeof(unsigned long long), hipHostMallocDefault));
    h->cap = cap;
  }
  for (size_t i = 0; i < J; ++i) {
    SampleArgs& a = subs[i]->a;
    if ((uint64_t)a.g.n > h->big_stride) return fail(TIM_EINVAL, "graph larger than the batch's slots");
    a.ctr = h->d_ctr + i * tim::kCtrCount;
    a.big_stamp = h->big_stamp;
    a.big_queue = h->big_queue;
    a.big_epoch = h->big_epoch;
    a.big_slots = h->big_slots;
    a.big_stride = h->big_stride;
    h->h_jobs[i] = a;
    HIP_TRY(hipStreamWaitEvent(h->stream, subs[i]->ready, 0));
  }
  HIP_TRY(hipMemcpyAsync(h->d_jobs, h->h_jobs, J * sizeof(SampleArgs), hipMemcpyHostToDevice, h->stream));
  tim::launch_clear_counters_batch(tim::JobTable{h->d_jobs, (int)J, 0}, h->stream);
  for (size_t lo = 0; lo < J;) {
    size_t hi = lo + 1;
    while (hi < J && cls(subs[hi]) == cls(subs[lo]) && hi - lo < (size_t)tim::kMaxBatchJobs) ++hi;
    const Pending* p = subs[lo];
    uint64_t total = 0, maxc = 0;
    for (size_t i = lo; i < hi; ++i) {
      total += subs[i]->a.count;
      maxc = std::max<uint64_t>(maxc, subs[i]->a.count);
    }
    const uint64_t per_block = p->model == TIM_MODEL_IC ? 32 : 128;  // sets a tier-0 block holds at once
    const uint64_t full = (uint64_t)h->grid0[p->model][p->mode][p->wc ? 1 : 0] * (uint64_t)h->num_cu;
    const uint64_t grid0 = std::max<uint64_t>(1, std::min(full, (total + per_block - 1) / per_block));
    const uint64_t grid1 =
        (uint64_t)(p->model == TIM_MODEL_IC ? h->grid1[p->mode][p->wc ? 1 : 0] : h->grid_chain[p->mode]) *
        (uint64_t)h->num_cu;
    const bool prof = h->owner && h->owner->prof_on;
    if (prof) HIP_TRY(hipEventRecord(h->pev[0], h->stream));
    tim::launch_sample_batch(p->model, p->mode, p->wc, tim::JobTable{h->d_jobs + lo, (int)(hi - lo), 0}, (int)grid0,
                             (int)grid1, h->big_slots, maxc, h->stream, prof ? h->pev[1] : nullptr);
    if (prof) {
      // the profile needs this launch's counters: wait for it
      HIP_TRY(hipEventRecord(h->pev[2], h->stream));
      HIP_TRY(hipMemcpyAsync(h->h_ctr + lo * tim::kCtrCount, h->d_ctr + lo * tim::kCtrCount,
                             (hi - lo) * tim::kCtrCount * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             h->stream));
      HIP_TRY(hipStreamSynchronize(h->stream));
      float ms_main = 0.f, ms_big = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms_main, h->pev[0], h->pev[1]));
      HIP_TRY(hipEventElapsedTime(&ms_big, h->pev[1], h->pev[2]));
      tim_kernel_profile& kp = h->owner->prof.sampler[p->model][p->mode];
      for (size_t i = lo; i < hi; ++i) {
        const unsigned long long* hc = h->h_ctr + i * tim::kCtrCount;
        const unsigned long long* acc0 = hc + tim::kCtrAcc;
        const uint64_t sets = subs[i]->a.count - hc[tim::kCtrList1];
        const uint64_t nodes = acc0[tim::kAccNodes], edges = acc0[tim::kAccWidth];
        uint64_t bytes = p->model == TIM_MODEL_IC ? 16 * nodes + (p->wc ? 4 : 8) * edges : 20 * nodes;
        if (p->mode == tim::kModeEmit) bytes += 4 * nodes + 12 * sets;
        kp.sets += sets;
        kp.nodes += nodes;
        kp.edges += edges;
        kp.bytes += bytes;
        kp.deferred += hc[tim::kCtrList1];
      }
      kp.launches += 1;
      kp.kernel_ms += ms_main;
      kp.large_launches += 1;
      kp.large_ms += ms_big;
    }
    h->launches += 1;
    lo = hi;
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(h->h_ctr, h->d_ctr, J * tim::kCtrCount * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                         h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (size_t i = 0; i < J; ++i)
    memcpy(subs[i]->h, h->h_ctr + i * tim::kCtrCount, sizeof(subs[i]->h));
  h->rounds += 1;
  h->jobs += J;
  h->max_jobs = std::max<uint64_t>(h->max_jobs, J);
  return TIM_OK;
}

void hub_scheduler(Hub* h) {
  (void)hipSetDevice(h->device);
  std::unique_lock<std::mutex> lk(h->mu);
  for (;;) {
    h->cv_sched.wait(lk, [&] { return h->stop || !h->waiting.empty(); });
    if (h->waiting.empty()) break;  // stop with nothing pending
    // gather until every worker still running waits, or the window has passed
    h->cv_sched.wait_until(lk, h->first_wait + h->window, [&] { return (int)h->waiting.size() >= h->alive; });
    std::vector<Pending*> subs;
    subs.swap(h->waiting);
    lk.unlock();
    const tim_status st = hub_round(h, subs);
    const std::string err = st == TIM_OK ? std::string() : g_error;
    lk.lock();
    for (Pending* p : subs) {
      p->st = st;
      p->err = err;
      p->done = true;
    }
    // requests that came in during the round get a fresh window, so that the
    // queries this round releases can join them
    if (!h->waiting.empty()) h->first_wait = std::chrono::steady_clock::now();
    h->cv_done.notify_all();
  }
}

void hub_enter(Hub* h) {
  std::lock_guard<std::mutex> lk(h->mu);
  h->alive += 1;
}

void hub_leave(Hub* h) {
  std::lock_guard<std::mutex> lk(h->mu);
  h->alive -= 1;
  h->cv_sched.notify_one();
}

// A member context of the hub: its own stream and buffers, and 8 lanes per
// IC set in tier 0 (the batched kernels' shape).
tim_status hub_member(Hub* h, const tim_ctx* parent, tim_ctx** out) {
  tim_ctx* c = nullptr;
  TIM_TRY(tim_ctx_create(parent->device, nullptr, 0, &c));
  c->hub = h;
  c->parent = parent;
  c->seg_lanes = 8;
  if (hipEventCreateWithFlags(&c->ready_ev, hipEventDisableTiming) != hipSuccess) {
    tim_ctx_destroy(c);
    return fail(TIM_EDEVICE, "hipEventCreate failed");
  }
  *out = c;
  return TIM_OK;
}

void batch_worker(Hub* h, tim_ctx* c, tim_query* qs, int nq, std::atomic<int>* next,
                  std::vector<std::string>* errs, const std::vector<tim_kpt_result>* kpts) {
  (void)hipSetDevice(c->device);
  for (;;) {
    const int i = next->fetch_add(1);
    if (i >= nq) break;
    tim_query& q = qs[i];
    q.status = run_impl(c, q.graph, q.model, q.k, q.eps, q.ell, q.seed, q.flags, q.seeds, q.gains, q.report,
                        kpts ? &(*kpts)[(size_t)i] : nullptr);
    if (q.status != TIM_OK) (*errs)[(size_t)i] = g_error;
  }
  c->stored.valid = false;
  hub_leave(h);
}

// The hub's stream and launch shapes (once per context).
tim_status hub_setup(Hub* h, tim_ctx* parent) {
  h->owner = parent;
  h->device = parent->device;
  h->num_cu = parent->num_cu;
  HIP_TRY(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
  for (hipEvent_t& e : h->pev) HIP_TRY(hipEventCreate(&e));
  for (int model = 0; model < 2; ++model)
    for (int mode = 0; mode < 3; ++mode)
      for (int wc = 0; wc < 2; ++wc) h->grid0[model][mode][wc] = tim::batch_blocks_per_cu(model, mode, wc != 0, 0);
  for (int mode = 0; mode < 3; ++mode)
    for (int wc = 0; wc < 2; ++wc) h->grid1[mode][wc] = tim::batch_blocks_per_cu(0, mode, wc != 0, 1);
  for (int mode = 0; mode < 3; ++mode) h->grid_chain[mode] = tim::lt_chain_blocks_per_cu(mode, true);
  h->emit_waves[0] = (uint64_t)std::max(h->grid0[0][1][0], h->grid0[0][1][1]) * (uint64_t)h->num_cu * 4;
  h->emit_waves[1] = (uint64_t)h->grid0[1][1][0] * (uint64_t)h->num_cu * 2;
  return TIM_OK;
}

void hub_free_slots(Hub* h) {
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  void* dev[] = {h->big_stamp, h->big_queue, h->big_epoch};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  h->big_stamp = nullptr;
  h->big_queue = nullptr;
  h->big_epoch = nullptr;
  h->big_slots = 0;
  h->big_stride = 0;
  h->big_bytes = 0;
}

// Memory of one call: the batch gets the context's budget less what the
// context itself holds (without a budget: 85% of the device memory that is
// free or already held by the hub and its members); the last-tier slots for
// the largest graph come first (one per CU where a quarter of it allows),
// and every query running at once gets an equal share of the rest.  Under a
// budget, the work buffers and last-tier slots that the context's own calls
// left are released first: the batch's members and hub have their own.
tim_status hub_prepare(Hub* h, tim_ctx* parent, int64_t maxn, int workers) {
  uint64_t limit = 0;
  if (parent->budget) {
    release_transients(parent);
    release(parent, parent->big_stamp);
    release(parent, parent->big_queue);
    release(parent, parent->big_epoch);
    parent->big_slots = 0;
    parent->big_n = -1;
    limit = parent->budget > parent->held ? parent->budget - parent->held : 0;
  } else {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    uint64_t ours = h->big_bytes;
    for (const tim_ctx* m : parent->members) ours += m->held;
    limit = (uint64_t)(0.85 * (double)(free_b + ours));
  }
  h->limit = limit;
  maxn = std::max<int64_t>(maxn, 2);
  const uint64_t per = (uint64_t)maxn * 8;
  // as ensure_big: one slot per CU, up to four while they take at most a sixteenth of the limit
  const int slots = (int)std::max(std::min<uint64_t>((uint64_t)std::max(h->num_cu, 64), limit / 4 / per),
                                  std::min<uint64_t>((uint64_t)std::max(4 * h->num_cu, 64), limit / 16 / per));
  if (slots < 1) return fail(TIM_EBUDGET, "budget too small for the large-set pass of the batch");
  // kept from an earlier batch unless too small for its graphs, or too large for this limit
  if (h->big_stride < (uint64_t)maxn || h->big_slots == 0 || h->big_bytes > limit / 4) {
    hub_free_slots(h);
    HIP_TRY(hipMalloc(&h->big_stamp, (size_t)slots * (size_t)maxn * 4));
    HIP_TRY(hipMalloc(&h->big_queue, (size_t)slots * (size_t)maxn * 4));
    HIP_TRY(hipMalloc(&h->big_epoch, (size_t)slots * 4));
    HIP_TRY(hipMemsetAsync(h->big_stamp, 0, (size_t)slots * (size_t)maxn * 4, h->stream));
    HIP_TRY(hipMemsetAsync(h->big_epoch, 0, (size_t)slots * 4, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->big_stride = (uint64_t)maxn;
    h->big_slots = slots;
    h->big_bytes = (uint64_t)slots * per + (uint64_t)slots * 4;
  }
  // half of what is left after the slots is shared equally among the queries running at once (their
  // KptEstimation and RefineKPT work space), the other half is the RR pool granted to NodeSelection
  const uint64_t rest = limit - std::min(limit, h->big_bytes);
  // a share holds at least the node-pool slices of one small stored-set launch (any wavefront of a
  // batched launch may reserve one in any job), the greedy's per-node arrays for the largest graph
  // and the lists of small launches
  uint64_t slices = 0;
  for (int model = 0; model < 2; ++model) {
    const uint64_t cap = tim::tier0_set_cap(model, 8);
    slices = std::max<uint64_t>(slices, h->emit_waves[model] * 5 * cap * 4);
  }
  const uint64_t min_share = 2 * slices + 17 * (uint64_t)maxn + (8u << 20);
  h->member_budget = std::max<uint64_t>(rest / 2 / (uint64_t)workers, min_share);
  if (h->member_budget * (uint64_t)workers >= rest)
    return fail(TIM_EBUDGET, "budget too small for %d queries at once (%llu bytes each and an RR pool)", workers,
                (unsigned long long)min_share);
  h->rr_total = rest - h->member_budget * (uint64_t)workers;
  if (const char* cap = getenv("TIM_RR_POOL_BYTES")) {  // a smaller RR pool than the budget allows
    const uint64_t v = strtoull(cap, nullptr, 10);
    if (v >= (1u << 20)) h->rr_total = std::min(h->rr_total, v);
  }
  h->rr_free = h->rr_total;
  h->rr_peak = 0;
  h->next_ticket = h->serving_ticket = 0;
  h->held = 0;
  h->held_ms = 0.0;
  while ((int)parent->members.size() < workers) {
    tim_ctx* m = nullptr;
    TIM_TRY(hub_member(h, parent, &m));
    parent->members.push_back(m);
  }
  for (int w = 0; w < workers; ++w) {
    tim_ctx* m = parent->members[(size_t)w];
    m->budget = h->member_budget;
    m->share = h->member_budget;
    m->resident_limit = parent->resident_limit;
    if (m->held > m->budget) release_transients(m);
  }
  // this call's state
  const char* env = getenv("TIM_BATCH_WINDOW_US");
  h->window = std::chrono::microseconds(env ? std::max(0L, atol(env)) : 1000L);
  h->waiting.clear();
  h->stop = false;
  h->alive = workers;
  h->rounds = h->jobs = h->launches = h->max_jobs = 0;
  h->kpt_steps = h->kpt_graph_launches = 0;
  return TIM_OK;
}

void hub_destroy(tim_ctx* parent) {
  for (tim_ctx* m : parent->members) tim_ctx_destroy(m);
  parent->members.clear();
  Hub* h = parent->batch;
  if (!h) return;
  hub_free_slots(h);
  void* dev[] = {h->d_jobs, h->d_ctr};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (h->h_jobs) (void)hipHostFree(h->h_jobs);
  if (h->h_ctr) (void)hipHostFree(h->h_ctr);
  for (hipEvent_t e : h->pev)
    if (e) (void)hipEventDestroy(e);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  parent->batch = nullptr;
}

// ---- batches: Algorithm 2 of every query on the device ----
//
// tim_run_batch first runs KptEstimation for all its queries without the
// host between rounds: per class of queries (model, thresholds), up to 64 at
// a time, a step hands each query a chunk of its current round (kpt_jobs),
// the batched samplers run the chunks (their wavefronts move from query to
// query), and kpt_advance adds the chunks' totals to their rounds and takes
// Algorithm 2's stop test where a round is complete.  kKptGraphSteps steps
// are captured as one HIP graph, replayed until no query is left; the host
// reads one flag per replay.  The queries' RefineKPT and NodeSelection then
// run as before (worker threads, the hub batching their sampling requests);
// R' of RefineKPT is generated again from its keys.
constexpr int kKptGraphSteps = 4;

// Sets in all per step: bounded by the batch's memory (20 bytes per set).
uint64_t kpt_step_cap(uint64_t limit) {
  return std::max<uint64_t>(1ull << 16, std::min<uint64_t>(1ull << 23, limit / 4 / 20));
}

tim_status batch_kpt_group(tim_ctx* c, Hub* h, tim_query* qs, const std::vector<int>& idx, int model, bool wc,
                           uint64_t job_cap, std::vector<tim_kpt_result>* out) {
  const int nq = (int)idx.size();
  std::vector<tim::KptQuery> hq((size_t)nq);
  std::vector<int> live;  // queries with at least one round
  for (int j = 0; j < nq; ++j) {
    const tim_query& q = qs[idx[(size_t)j]];
    const tim_graph* g = q.graph;
    tim_kpt_result& r = (*out)[(size_t)idx[(size_t)j]];
    memset(&r, 0, sizeof(r));
    const int imax = rounds_of(g->n);
    r.i_max = imax;
    r.i_last = imax;
    r.c_last = imax >= 1 ? round_size(g->n, ell_of(g, q.ell, q.flags), imax) : 0;
    r.kpt_star = 1.0;
    tim::KptQuery& d = hq[(size_t)j];
    memset(&d, 0, sizeof(d));
    d.g.off = g->off;
    d.g.off32 = g->off32;
    d.g.src = g->src;
    d.g.thr = g->thr;
    d.g.lthr = g->lthr;
    d.g.n = g->n;
    d.g.m = g->m;
    d.seed = q.seed;
    d.k = q.k;
    d.imax = imax;
    d.round = imax >= 1 ? 1 : 0;
    d.i_last = imax;
    for (int i = 1; i <= imax && i < tim::kKptMaxRounds; ++i) d.c[i] = round_size(g->n, ell_of(g, q.ell, q.flags), i);
  }
  const uint64_t step_cap = kpt_step_cap(h->limit > h->big_bytes ? h->limit - h->big_bytes : 0);
  TIM_TRY(ensure(c, c->wbuf, step_cap * 4, "width buffer"));
  TIM_TRY(ensure(c, c->list1, step_cap * 8, "deferred-set list"));
  if (model == TIM_MODEL_IC) TIM_TRY(ensure(c, c->list2, step_cap * 8, "deferred-set list"));
  const size_t qbytes = ((size_t)nq * sizeof(tim::KptQuery) + 255) & ~(size_t)255;
  const size_t jbytes = ((size_t)nq * sizeof(SampleArgs) + 255) & ~(size_t)255;
  const size_t cbytes = (size_t)nq * tim::kCtrCount * 8;
  TIM_TRY(ensure(c, c->jobs, qbytes + jbytes + cbytes + 256, "batch KptEstimation state"));
  char* base = static_cast<char*>(c->jobs.p);
  tim::KptStepArgs a;
  memset(&a, 0, sizeof(a));
  a.q = reinterpret_cast<tim::KptQuery*>(base);
  a.nq = nq;
  a.jobs = reinterpret_cast<SampleArgs*>(base + qbytes);
  a.ctr = reinterpret_cast<unsigned long long*>(base + qbytes + jbytes);
  a.active = reinterpret_cast<unsigned int*>(base + qbytes + jbytes + cbytes);
  a.wbuf = c->wbuf.as<uint32_t>();
  a.list1 = c->list1.as<uint64_t>();
  a.list2 = model == TIM_MODEL_IC ? c->list2.as<uint64_t>() : nullptr;
  a.step_cap = step_cap;
  a.job_cap = std::max<uint64_t>(1, job_cap);
  a.big_stamp = h->big_stamp;
  a.big_queue = h->big_queue;
  a.big_epoch = h->big_epoch;
  a.big_slots = h->big_slots;
  a.big_stride = h->big_stride;
  HIP_TRY(hipMemcpyAsync(a.q, hq.data(), (size_t)nq * sizeof(tim::KptQuery), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));

  // the steps, captured once as a graph
  const tim::JobTable tab{a.jobs, nq, 0};
  const int mode = tim::kModeWidth;
  const uint64_t grid0 = (uint64_t)h->grid0[model][mode][wc ? 1 : 0] * (uint64_t)h->num_cu;
  const uint64_t grid1 =
      (uint64_t)(model == TIM_MODEL_IC ? h->grid1[mode][wc ? 1 : 0] : h->grid_chain[mode]) * (uint64_t)h->num_cu;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  for (int st = 0; st < kKptGraphSteps; ++st) {
    tim::launch_kpt_jobs(a, h->stream);
    tim::launch_clear_counters_batch(tab, h->stream);
    tim::launch_sample_batch(model, mode, wc, tab, (int)grid0, (int)grid1, h->big_slots, step_cap, h->stream, nullptr);
    tim::launch_kpt_advance(a, h->stream);
  }
  const hipError_t ce = hipStreamEndCapture(h->stream, &graph);
  if (ce != hipSuccess) return fail(TIM_EDEVICE, "capture of the KptEstimation steps: %s", hipGetErrorString(ce));
  struct GraphScope {
    hipGraph_t g;
    hipGraphExec_t e;
    ~GraphScope() {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
    }
  } scope{graph, nullptr};
  HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  scope.e = exec;
  unsigned int* active_host = reinterpret_cast<unsigned int*>(c->ctr_host);
  for (int launches = 0;; ++launches) {
    if (launches > 1 << 16) return fail(TIM_EDEVICE, "batch KptEstimation did not finish");
    HIP_TRY(hipGraphLaunch(exec, h->stream));
    HIP_TRY(hipMemcpyAsync(active_host, a.active, 4, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->kpt_steps += kKptGraphSteps;
    h->kpt_graph_launches += 1;
    if (*active_host == 0u) break;
  }
  HIP_TRY(hipMemcpyAsync(hq.data(), a.q, (size_t)nq * sizeof(tim::KptQuery), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int j = 0; j < nq; ++j) {
    const tim::KptQuery& d = hq[(size_t)j];
    if (d.err) return fail(TIM_EDEVICE, "deferred-set list overflow");
    tim_kpt_result& r = (*out)[(size_t)idx[(size_t)j]];
    if (d.imax < 1) continue;
    r.i_last = d.i_last;
    r.c_last = d.c[d.i_last];
    for (int i = 1; i <= d.i_last; ++i) {
      r.round_c[i] = d.c[i];
      r.round_sum_lo[i] = d.r_lo[i];
      r.round_sum_hi[i] = d.r_hi[i];
      r.round_width[i] = d.r_width[i];
      r.round_nodes[i] = d.r_nodes[i];
    }
    kpt_finish_result(qs[idx[(size_t)j]].graph, &r);
  }
  return TIM_OK;
}

// Algorithm 2 for every query of a batch on the device, by classes of up to 64.
tim_status batch_kpt(tim_ctx* c, Hub* h, tim_query* qs, int count, uint64_t job_cap,
                     std::vector<tim_kpt_result>* out) {
  out->assign((size_t)count, tim_kpt_result());
  std::vector<int> cls[2][2];
  for (int i = 0; i < count; ++i) {
    const tim_query& q = qs[i];
    const bool wc = q.model != TIM_MODEL_IC || q.graph->thr == nullptr;
    cls[q.model][wc ? 1 : 0].push_back(i);
  }
  for (int model = 0; model < 2; ++model)
    for (int wc = 0; wc < 2; ++wc)
      for (size_t lo = 0; lo < cls[model][wc].size(); lo += tim::kMaxBatchJobs) {
        const size_t hi = std::min(cls[model][wc].size(), lo + (size_t)tim::kMaxBatchJobs);
        std::vector<int> idx(cls[model][wc].begin() + (long)lo, cls[model][wc].begin() + (long)hi);
        TIM_TRY(batch_kpt_group(c, h, qs, idx, model, wc != 0, job_cap, out));
      }
  for (DevBuf* b : {&c->list1, &c->list2, &c->wbuf, &c->jobs}) release(c, *b);
  return TIM_OK;
}

// ---- serving: queries that arrive over time ----
//
// The same hub and member contexts as a batch.  Submitted queries wait in a
// queue; each of `slots` worker threads takes the next one when it is free
// and runs it on its member context.  The hub's rounds gather the sampling
// requests of whichever queries are running at that moment (continuous
// batching): a query that arrives while others are on the GPU joins the
// next round its worker reaches.

struct Ticket {
  tim_query* q = nullptr;
  std::chrono::steady_clock::time_point submitted, finished;
  bool done = false;
  std::string err;
};

}  // namespace

struct tim_server {
  tim_ctx* ctx = nullptr;
  Hub* hub = nullptr;
  int slots = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<Ticket*> queue;  // FIFO: queue[head ..]
  size_t head = 0;
  std::vector<Ticket*> tickets;  // by ticket number
  bool stopping = false;
  std::vector<std::thread> workers;
  std::thread sched;
};

namespace {

void server_worker(tim_server* sv, tim_ctx* c) {
  (void)hipSetDevice(c->device);
  for (;;) {
    Ticket* t = nullptr;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] { return sv->stopping || sv->head < sv->queue.size(); });
      if (sv->head == sv->queue.size()) break;  // stopping, nothing left
      t = sv->queue[sv->head++];
    }
    hub_enter(sv->hub);
    tim_query& q = *t->q;
    q.status = run_impl(c, q.graph, q.model, q.k, q.eps, q.ell, q.seed, q.flags, q.seeds, q.gains, q.report);
    const std::string err = q.status == TIM_OK ? std::string() : g_error;
    c->stored.valid = false;
    hub_leave(sv->hub);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      t->err = err;
      t->finished = std::chrono::steady_clock::now();
      t->done = true;
    }
    sv->cv_done.notify_all();
  }
}

}  // namespace

// =========================================================================
// C ABI
// =========================================================================
extern "C" {

const char* tim_last_error(void) { return g_error.c_str(); }

tim_status tim_ctx_create(int device, void* stream, uint64_t hbm_budget_bytes, tim_ctx** out) {
  if (!out) return fail(TIM_EINVAL, "out is null");
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(TIM_EDEVICE, "device %d not present (%d devices)", device, ndev);
  HIP_TRY(hipSetDevice(device));
  tim_ctx* c = new tim_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return fail(TIM_EDEVICE, "hipGetDeviceProperties failed");
  }
  c->num_cu = prop.multiProcessorCount;
  if (stream) {
    c->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(TIM_EDEVICE, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  c->seg_lanes = tim::ic_seg_lanes();
  for (int mode = 0; mode < 3; ++mode) {
    for (int wc = 0; wc < 2; ++wc) {
      c->grid_ic[mode][wc] = tim::ic_blocks_per_cu(mode, wc != 0, c->seg_lanes);
      c->grid_ic64[mode][wc] = tim::ic_tier1_blocks_per_cu(mode, wc != 0);
      c->grid_ic_wide[mode][wc] = tim::ic_blocks_per_cu(mode, wc != 0, 64);
    }
    c->grid_lt[mode] = tim::lt_lane_blocks_per_cu(mode);
    c->grid_trig[mode] = tim::trig_blocks_per_cu(mode);
    c->grid_trig1[mode] = tim::trig_tier1_blocks_per_cu(mode);
    c->grid_lt_chain[mode] = tim::lt_chain_blocks_per_cu(mode, false);
  }
  for (int wc = 0; wc < 2; ++wc) {
    for (int model = 0; model < 2; ++model)
      c->grid_rounds[model][wc] = tim::batch_blocks_per_cu(model, tim::kModeWidth, wc != 0, 0);
    c->grid_batch1[wc] = tim::batch_blocks_per_cu(0, tim::kModeWidth, wc != 0, 1);
  }
  c->grid_batch_chain = tim::lt_chain_blocks_per_cu(tim::kModeWidth, true);
  {
    // the fixed work area of tim_max_coverage_noalloc on this device (once per device)
    const hipError_t e = tim::static_scratch_init(device);
    if (e != hipSuccess) {
      if (c->own_stream) (void)hipStreamDestroy(c->stream);
      delete c;
      return fail(TIM_EDEVICE, "hipGetSymbolAddress of the fixed work area: %s", hipGetErrorString(e));
    }
  }
  if (hipMalloc(&c->ctr, tim::kCtrCount * sizeof(unsigned long long)) != hipSuccess ||
      hipHostMalloc(&c->ctr_host, tim::kCtrCount * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess ||
      hipEventCreate(&c->pev[0]) != hipSuccess || hipEventCreate(&c->pev[1]) != hipSuccess ||
      hipEventCreate(&c->pev[2]) != hipSuccess) {
    tim_ctx_destroy(c);
    return fail(TIM_EDEVICE, "context allocation failed");
  }
  *out = c;
  return TIM_OK;
}

void tim_ctx_destroy(tim_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  hub_destroy(c);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  DevBuf* bufs[] = {&c->list1, &c->list2, &c->wbuf, &c->pool, &c->set_start, &c->set_len, &c->big_stamp, &c->big_queue, &c->big_epoch,
                    &c->rr_off, &c->rr_nodes, &c->sizes, &c->cnt, &c->fill, &c->inv_off, &c->inv_sets, &c->covered,
                    &c->selected, &c->best, &c->scan_tmp, &c->bucket, &c->seed_bits, &c->jobs};
  for (DevBuf* b : bufs) release(c, *b);
  if (c->ctr) (void)hipFree(c->ctr);
  if (c->ctr_host) (void)hipHostFree(c->ctr_host);
  for (hipEvent_t e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->pev)
    if (e) (void)hipEventDestroy(e);
  if (c->ready_ev) (void)hipEventDestroy(c->ready_ev);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

uint64_t tim_ctx_device_bytes(const tim_ctx* c) { return c ? c->held : 0; }

tim_status tim_set_resident_limit(tim_ctx* c, uint64_t max_sets) {
  if (!c) return fail(TIM_EINVAL, "null context");
  c->resident_limit = max_sets;
  return TIM_OK;
}

tim_status tim_profile_enable(tim_ctx* c, int on) {
  if (!c) return fail(TIM_EINVAL, "null context");
  c->prof_on = on != 0;
  memset(&c->prof, 0, sizeof(c->prof));
  return TIM_OK;
}

tim_status tim_profile_read(const tim_ctx* c, tim_profile* out) {
  if (!c || !out) return fail(TIM_EINVAL, "null argument");
  *out = c->prof;
  return TIM_OK;
}

tim_status tim_graph_upload(tim_ctx* c, int64_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                            const uint32_t* ic_thr, tim_graph** out) {
  if (!c || !out || !in_off || !in_src) return fail(TIM_EINVAL, "null argument");
  *out = nullptr;
  if (n < 2 || n > 0x7FFFFFFFLL) return fail(TIM_EINVAL, "n=%lld outside [2, 2^31)", (long long)n);
  if (m < 1 || m > 0xFFFFFFF0LL) return fail(TIM_EINVAL, "m=%lld outside [1, 2^32 - 16]", (long long)m);
  if (in_off[0] != 0 || in_off[n] != m) return fail(TIM_EINVAL, "in_off[0] must be 0 and in_off[n] must be m");
  for (int64_t v = 0; v < n; ++v) {
    if (in_off[v + 1] < in_off[v]) return fail(TIM_EINVAL, "in_off decreases at node %lld", (long long)v);
    for (int64_t e = in_off[v]; e < in_off[v + 1]; ++e) {
      const int32_t u = in_src[e];
      if (u < 0 || u >= n) return fail(TIM_EINVAL, "source of edge %lld out of range", (long long)e);
      if (u == v) return fail(TIM_EINVAL, "self-loop at node %lld", (long long)v);
      if (e > in_off[v] && in_src[e - 1] >= u)
        return fail(TIM_EINVAL, "in-edges of node %lld not strictly increasing by source", (long long)v);
    }
  }
  HIP_TRY(hipSetDevice(c->device));
  tim_graph* g = new tim_graph();
  g->ctx = c;
  c->max_graph_n = std::max<int64_t>(c->max_graph_n, n);
  g->n = n;
  g->m = m;
  const size_t mpad = (size_t)((m + 3) / 4 * 4 + 4);
  std::vector<uint32_t> off32((size_t)n + 1);
  for (int64_t v = 0; v <= n; ++v) off32[(size_t)v] = (uint32_t)in_off[v];  // m < 2^32
  bool ok = hipMalloc(&g->off, (size_t)(n + 1) * 8) == hipSuccess &&
            hipMalloc(&g->off32, (size_t)(n + 1) * 4) == hipSuccess && hipMalloc(&g->src, mpad * 4) == hipSuccess &&
            (!ic_thr || hipMalloc(&g->thr, mpad * 4) == hipSuccess);
  if (ok) {
    ok = hipMemcpyAsync(g->off, in_off, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
         hipMemcpyAsync(g->off32, off32.data(), (size_t)(n + 1) * 4, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
         hipMemsetAsync(g->src, 0, mpad * 4, c->stream) == hipSuccess &&
         hipMemcpyAsync(g->src, in_src, (size_t)m * 4, hipMemcpyHostToDevice, c->stream) == hipSuccess;
    if (ok && ic_thr)
      ok = hipMemsetAsync(g->thr, 0, mpad * 4, c->stream) == hipSuccess &&
           hipMemcpyAsync(g->thr, ic_thr, (size_t)m * 4, hipMemcpyHostToDevice, c->stream) == hipSuccess;
    ok = ok && hipStreamSynchronize(c->stream) == hipSuccess;
  }
  if (!ok) {
    tim_graph_free(g);
    return fail(TIM_ENOMEM, "graph upload failed");
  }
  *out = g;
  return TIM_OK;
}

void tim_graph_free(tim_graph* g) {
  if (!g) return;
  if (g->off) (void)hipFree(g->off);
  if (g->off32) (void)hipFree(g->off32);
  if (g->src) (void)hipFree(g->src);
  if (g->thr) (void)hipFree(g->thr);
  if (g->lthr) (void)hipFree(g->lthr);
  for (void* p : {(void*)g->toff, (void*)g->tthr, (void*)g->tset, (void*)g->tmem})
    if (p) (void)hipFree(p);
  if (g->out_off) (void)hipFree(g->out_off);
  if (g->out_dst) (void)hipFree(g->out_dst);
  if (g->out_eid) (void)hipFree(g->out_eid);
  delete g;
}

tim_status tim_graph_set_lt_weights(tim_ctx* c, tim_graph* g, const uint32_t* lt_thr, const int64_t* in_off) {
  if (!c || !g || g->ctx != c) return fail(TIM_EINVAL, "graph does not belong to this context");
  if (c->serving) return fail(TIM_EINVAL, "a server runs on this context");
  HIP_TRY(hipSetDevice(c->device));
  if (!lt_thr) {
    if (g->lthr) {
      HIP_TRY(hipStreamSynchronize(c->stream));
      (void)hipFree(g->lthr);
    }
    g->lthr = nullptr;
    return TIM_OK;
  }
  if (!in_off) return fail(TIM_EINVAL, "in_off is null");
  if (in_off[0] != 0 || in_off[g->n] != g->m) return fail(TIM_EINVAL, "in_off does not match the graph");
  for (int64_t v = 0; v < g->n; ++v)
    for (int64_t e = in_off[v] + 1; e < in_off[v + 1]; ++e)
      if (lt_thr[e] < lt_thr[e - 1])
        return fail(TIM_EINVAL, "LT thresholds of node %lld decrease at edge %lld", (long long)v, (long long)e);
  uint32_t* d = nullptr;
  if (hipMalloc(&d, (size_t)g->m * 4) != hipSuccess) return fail(TIM_ENOMEM, "LT thresholds: hipMalloc failed");
  if (hipMemcpyAsync(d, lt_thr, (size_t)g->m * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipFree(d);
    return fail(TIM_EDEVICE, "LT thresholds: copy failed");
  }
  if (g->lthr) (void)hipFree(g->lthr);
  g->lthr = d;
  return TIM_OK;
}

tim_status tim_graph_set_triggering(tim_ctx* c, tim_graph* g, const int64_t* toff, const uint32_t* tthr,
                                    const int64_t* tset, const uint32_t* tmem, const int64_t* in_off) {
  if (!c || !g || g->ctx != c) return fail(TIM_EINVAL, "graph does not belong to this context");
  if (c->serving) return fail(TIM_EINVAL, "a server runs on this context");
  HIP_TRY(hipSetDevice(c->device));
  auto drop = [&]() {
    for (void** p : {(void**)&g->toff, (void**)&g->tthr, (void**)&g->tset, (void**)&g->tmem}) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
  };
  if (!toff) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    drop();
    return TIM_OK;
  }
  if (!tthr || !tset || !tmem || !in_off) return fail(TIM_EINVAL, "null argument");
  if (in_off[0] != 0 || in_off[g->n] != g->m) return fail(TIM_EINVAL, "in_off does not match the graph");
  if (toff[0] != 0) return fail(TIM_EINVAL, "toff[0] must be 0");
  for (int64_t v = 0; v < g->n; ++v)
    if (toff[v + 1] < toff[v]) return fail(TIM_EINVAL, "toff decreases at node %lld", (long long)v);
  const int64_t J = toff[g->n];
  if (J > 0xFFFFFFFFLL) return fail(TIM_EINVAL, "more than 2^32 - 1 outcomes");
  if (tset[0] != 0) return fail(TIM_EINVAL, "tset[0] must be 0");
  for (int64_t j = 0; j < J; ++j)
    if (tset[j + 1] < tset[j]) return fail(TIM_EINVAL, "tset decreases at outcome %lld", (long long)j);
  const int64_t total = tset[J];
  for (int64_t v = 0; v < g->n; ++v) {
    const int64_t d = in_off[v + 1] - in_off[v];
    for (int64_t j = toff[v]; j < toff[v + 1]; ++j) {
      if (j > toff[v] && tthr[j] < tthr[j - 1])
        return fail(TIM_EINVAL, "thresholds of node %lld decrease at outcome %lld", (long long)v, (long long)j);
      for (int64_t i = tset[j]; i < tset[j + 1]; ++i) {
        if ((int64_t)tmem[i] >= d)
          return fail(TIM_EINVAL, "member %lld of outcome %lld is not an in-edge of node %lld", (long long)i,
                      (long long)j, (long long)v);
        if (i > tset[j] && tmem[i] <= tmem[i - 1])
          return fail(TIM_EINVAL, "members of outcome %lld are not strictly increasing", (long long)j);
      }
    }
  }
  int64_t* d_off = nullptr;
  uint32_t* d_thr = nullptr;
  int64_t* d_set = nullptr;
  uint32_t* d_mem = nullptr;
  bool ok = hipMalloc(&d_off, (size_t)(g->n + 1) * 8) == hipSuccess &&
            hipMalloc(&d_thr, (size_t)std::max<int64_t>(J, 1) * 4) == hipSuccess &&
            hipMalloc(&d_set, (size_t)(J + 1) * 8) == hipSuccess &&
            hipMalloc(&d_mem, (size_t)std::max<int64_t>(total, 1) * 4) == hipSuccess;
  if (ok)
    ok = hipMemcpyAsync(d_off, toff, (size_t)(g->n + 1) * 8, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
         (J == 0 || hipMemcpyAsync(d_thr, tthr, (size_t)J * 4, hipMemcpyHostToDevice, c->stream) == hipSuccess) &&
         hipMemcpyAsync(d_set, tset, (size_t)(J + 1) * 8, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
         (total == 0 ||
          hipMemcpyAsync(d_mem, tmem, (size_t)total * 4, hipMemcpyHostToDevice, c->stream) == hipSuccess) &&
         hipStreamSynchronize(c->stream) == hipSuccess;
  if (!ok) {
    for (void* p : {(void*)d_off, (void*)d_thr, (void*)d_set, (void*)d_mem})
      if (p) (void)hipFree(p);
    (void)hipGetLastError();
    return fail(TIM_ENOMEM, "triggering distribution: upload failed");
  }
  drop();
  g->toff = d_off;
  g->tthr = d_thr;
  g->tset = d_set;
  g->tmem = d_mem;
  return TIM_OK;
}

tim_status tim_sample_rr(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, uint32_t phase, uint64_t first,
                         uint64_t count, int64_t* d_set_off, int32_t* d_nodes, uint64_t nodes_capacity,
                         uint64_t* d_widths, uint64_t* total_nodes, tim_batch_stats* stats) {
  TIM_TRY(check_phase_args(c, g, model, 1));
  if (!d_set_off || phase > 255) return fail(TIM_EINVAL, "bad output offsets pointer or phase");
  HIP_TRY(hipSetDevice(c->device));
  Totals t;
  TIM_TRY(emit_sets(c, g, model, seed, phase, first, count, count * 16, d_widths, &t));
  if (total_nodes) *total_nodes = t.nodes;
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->count = count;
    stats->width_sum = t.width;
    stats->node_sum = t.nodes;
    stats->deferred = t.deferred;
  }
  TIM_TRY(ensure(c, c->scan_tmp, tim::scan_temp_bytes(count), "scan"));
  tim::launch_scan_u32_to_i64(c->set_len.as<uint32_t>(), d_set_off, count, c->scan_tmp.p, c->stream);
  if (t.nodes > nodes_capacity) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    return fail(TIM_ECAPACITY, "%llu nodes do not fit a buffer of %llu", (unsigned long long)t.nodes,
                (unsigned long long)nodes_capacity);
  }
  if (t.nodes && !d_nodes) return fail(TIM_EINVAL, "d_nodes is null");
  tim::launch_compact(c->pool.as<int32_t>(), c->set_start.as<uint64_t>(), c->set_len.as<uint32_t>(), d_set_off,
                      d_nodes, count, c->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(c->stream));
  return TIM_OK;
}

tim_status tim_sample_widths(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, uint32_t phase, uint64_t first,
                             uint64_t count, int k, uint64_t* d_widths, uint32_t* d_sizes, tim_batch_stats* stats) {
  TIM_TRY(check_phase_args(c, g, model, k));
  if (phase > 255) return fail(TIM_EINVAL, "phase %u > 255", phase);
  HIP_TRY(hipSetDevice(c->device));
  Totals t;
  TIM_TRY(sample_counts(c, g, model, tim::kModeWidth, seed, phase, first, count, k, d_widths, d_sizes, &t));
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->count = count;
    stats->kappa_sum_lo = (uint64_t)t.kappa;
    stats->kappa_sum_hi = (uint64_t)(t.kappa >> 64);
    stats->width_sum = t.width;
    stats->node_sum = t.nodes;
    stats->deferred = t.deferred;
  }
  return TIM_OK;
}

tim_status tim_sample_cover(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, uint32_t phase, uint64_t first,
                            uint64_t count, const int32_t* seeds, int nseeds, tim_batch_stats* stats) {
  TIM_TRY(check_phase_args(c, g, model, 1));
  if (phase > 255 || nseeds < 0 || (nseeds > 0 && !seeds)) return fail(TIM_EINVAL, "bad phase or seed list");
  HIP_TRY(hipSetDevice(c->device));
  TIM_TRY(upload_seed_bits(c, g->n, seeds, nseeds));
  Totals t;
  TIM_TRY(sample_counts(c, g, model, tim::kModeCover, seed, phase, first, count, 0, nullptr, nullptr, &t));
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->count = count;
    stats->covered = t.covered;
    stats->deferred = t.deferred;
  }
  return TIM_OK;
}

tim_status tim_max_coverage(tim_ctx* c, int64_t n, uint64_t nsets, const int64_t* d_set_off, const int32_t* d_nodes,
                            int k, int32_t* seeds, uint64_t* gains) {
  if (!c || !seeds || (nsets && (!d_set_off || !d_nodes))) return fail(TIM_EINVAL, "null argument");
  if (n < 1 || n > 0x7FFFFFFFLL || k < 1 || k > n) return fail(TIM_EINVAL, "bad n or k");
  HIP_TRY(hipSetDevice(c->device));
  int64_t total = 0;
  if (nsets) {
    HIP_TRY(hipMemcpyAsync(&total, d_set_off + nsets, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  if (total < 0) return fail(TIM_EINVAL, "negative collection size");
  if (total) {
    TIM_TRY(ensure(c, c->fill, 16, "id check flag"));
    tim::launch_check_ids(d_nodes, (uint64_t)total, n, c->fill.as<unsigned int>(), c->stream);
    unsigned int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, c->fill.p, 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (bad) return fail(TIM_EINVAL, "a node id of the collection lies outside [0, n)");
  }
  int64_t zero_off = 0;
  const int64_t* off = d_set_off;
  if (!nsets) {
    TIM_TRY(ensure(c, c->rr_off, 8, "empty offsets"));
    HIP_TRY(hipMemcpyAsync(c->rr_off.p, &zero_off, 8, hipMemcpyHostToDevice, c->stream));
    off = c->rr_off.as<int64_t>();
  }
  return greedy(c, n, nsets, off, nullptr, nullptr, d_nodes, (uint64_t)total, k, seeds, gains);
}

tim_status tim_max_coverage_noalloc(tim_ctx* c, int64_t n, uint64_t nsets, const int64_t* d_set_off,
                                    const int32_t* d_nodes, int k, int32_t* seeds, uint64_t* gains) {
  if (!c || !seeds || (nsets && (!d_set_off || !d_nodes))) return fail(TIM_EINVAL, "null argument");
  if (n < 1 || n > tim::kStaticMaxN || k < 1 || k > n || k > tim::kStaticMaxK)
    return fail(TIM_EINVAL, "n = %lld and k = %d must satisfy 1 <= k <= n, n <= %lld, k <= %d", (long long)n, k,
                (long long)tim::kStaticMaxN, tim::kStaticMaxK);
  if (nsets > tim::kStaticMaxSets)
    return fail(TIM_EINVAL, "%llu sets exceed the fixed work area's %llu", (unsigned long long)nsets,
                (unsigned long long)tim::kStaticMaxSets);
  HIP_TRY(hipSetDevice(c->device));
  const tim::StaticGreedy st = tim::static_greedy_layout(c->device);
  if (!st.cnt) return fail(TIM_EDEVICE, "the fixed work area of device %d was not set up", c->device);
  int64_t total = 0;
  if (nsets) {
    HIP_TRY(hipMemcpyAsync(&total, d_set_off + nsets, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  if (total < 0) return fail(TIM_EINVAL, "negative collection size");
  if ((uint64_t)total > tim::kStaticMaxEntries)
    return fail(TIM_EINVAL, "%lld entries exceed the fixed work area's %llu", (long long)total,
                (unsigned long long)tim::kStaticMaxEntries);
  if (total) {
    tim::launch_check_ids(d_nodes, (uint64_t)total, n, st.flag, c->stream);
    unsigned int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, st.flag, 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (bad) return fail(TIM_EINVAL, "a node id of the collection lies outside [0, n)");
  }
  const int64_t* off = d_set_off;
  if (!nsets) {
    tim::launch_set_u64(reinterpret_cast<unsigned long long*>(st.zero_off), 0ull, c->stream);
    off = st.zero_off;
  }
  tim::GreedyArgs a;
  memset(&a, 0, sizeof(a));
  a.n = n;
  a.nsets = nsets;
  a.total = (uint64_t)total;
  a.set_off = off;
  a.nodes = d_nodes;
  a.cnt = st.cnt;
  a.fill = st.fill;
  a.inv_off = st.inv_off;
  a.inv_sets = st.inv_sets;
  a.scan_temp = st.scan_temp;
  a.covered = st.covered;
  a.selected = st.selected;
  a.best = st.best;
  if (k > 1) tim::launch_index(a, c->stream);
  else tim::launch_counts(a, c->stream);
  tim::launch_greedy(a, k, c->stream);
  HIP_TRY(hipGetLastError());
  unsigned long long keys[tim::kStaticMaxK];
  HIP_TRY(hipMemcpyAsync(keys, a.best, (size_t)k * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int j = 0; j < k; ++j) {
    seeds[j] = (int32_t)(0xFFFFFFFFull - (keys[j] & 0xFFFFFFFFull));
    if (gains) gains[j] = keys[j] >> 32;
  }
  return TIM_OK;
}

tim_status tim_kpt_estimate(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, int k, double ell,
                            tim_kpt_result* out) {
  TIM_TRY(check_phase_args(c, g, model, k));
  if (!out || !(ell >= 0.5)) return fail(TIM_EINVAL, "ell must be >= 0.5");
  HIP_TRY(hipSetDevice(c->device));
  return kpt_estimate_impl(c, g, model, seed, k, ell, false, out, nullptr, nullptr);
}

tim_status tim_refine_kpt(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, int k, double eps, double ell,
                          double kpt_star, int i_last, uint64_t c_last, int32_t* s_prime, tim_refine_result* out) {
  TIM_TRY(check_phase_args(c, g, model, k));
  if (!s_prime || !out) return fail(TIM_EINVAL, "null output");
  if (!(eps > 0.0 && eps <= 1.0)) return fail(TIM_EINVAL, "eps must be in (0, 1]");
  if (!(ell >= 0.5) || !(kpt_star >= 1.0) || i_last < 0 || i_last > 62)
    return fail(TIM_EINVAL, "bad ell, KPT* or round");
  HIP_TRY(hipSetDevice(c->device));
  return refine_impl(c, g, model, seed, k, eps, ell, kpt_star, i_last, c_last, c_last * 16, s_prime, out, nullptr,
                     nullptr);
}

tim_status tim_node_select(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, int k, uint64_t theta,
                           int32_t* seeds, uint64_t* gains, tim_select_result* out) {
  TIM_TRY(check_phase_args(c, g, model, k));
  if (!seeds) return fail(TIM_EINVAL, "seeds is null");
  HIP_TRY(hipSetDevice(c->device));
  return node_select_impl(c, g, model, seed, k, theta, theta * 16, seeds, gains, out, nullptr);
}

tim_status tim_autotune(tim_ctx* c, const tim_graph* g, int model, uint64_t sets, tim_tune_result* out) {
  TIM_TRY(check_phase_args(c, g, model, 1));
  if (c->hub || c->serving) return fail(TIM_EINVAL, "context is a batch member or runs a server");
  if (model == TIM_MODEL_TRIGGER) return fail(TIM_EINVAL, "tim_autotune times the IC and LT samplers only");
  if (sets < 4096 || sets > kMaxLaunchSets) return fail(TIM_EINVAL, "sets must lie in [4096, 2^26]");
  HIP_TRY(hipSetDevice(c->device));
  tim_tune_result r;
  memset(&r, 0, sizeof(r));
  c->stored.valid = false;
  const uint64_t seed = 0x74756e65ull;  // the tuning sets are timed and dropped
  const uint32_t phase = 66;
  // best of three timed launches after one untimed; a failing launch leaves its status in st
  tim_status st = TIM_OK;
  auto best_ms = [&](auto&& launch) -> double {
    double best = 1e300;
    for (int trial = 0; trial < 4; ++trial) {
      const auto t0 = std::chrono::steady_clock::now();
      st = launch();
      if (st != TIM_OK) return -1.0;
      const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (trial > 0) best = std::min(best, ms);
    }
    return best;
  };
  // a candidate replaces the current shape only if it is at least 3% faster (timing noise)
  const double kGain = 0.97;
  uint64_t nodes = 0;
  if (model == TIM_MODEL_IC) {
    // every trial runs the shape it times, whatever the size of the trial launch
    struct WideScope {
      tim_ctx* c;
      ~WideScope() { c->wide_small = true; }
    } wide_scope{c};
    c->wide_small = false;
    static const int lanes[5] = {4, 8, 16, 32, 64};
    const int cur_lanes = c->seg_lanes;
    int best_lanes = cur_lanes;
    double best = 1e300, cur = 1e300;
    // a TIM+ run samples width-only rounds and stored sets: each shape is timed on one launch of each
    for (int i = 0; i < 5; ++i) {
      set_seg_lanes(c, lanes[i]);
      Totals t;
      const double ms_w = best_ms([&] {
        t = Totals();
        return sample_counts(c, g, model, tim::kModeWidth, seed, phase, 0, sets, 1, nullptr, nullptr, &t);
      });
      nodes = t.nodes;
      const double ms_e = ms_w < 0 ? -1.0 : best_ms([&] {
        Totals te;
        return emit_sets(c, g, model, seed, phase, 0, sets, nodes + nodes / 4 + 4096, nullptr, &te);
      });
      if (ms_w < 0 || ms_e < 0) {
        set_seg_lanes(c, best_lanes);
        return st;
      }
      r.ms_width[i] = ms_w;
      r.ms_lanes_emit[i] = ms_e;
      const double ms = ms_w + ms_e;
      if (lanes[i] == cur_lanes) cur = ms;
      if (ms < best) {
        best = ms;
        best_lanes = lanes[i];
      }
    }
    set_seg_lanes(c, best < kGain * cur ? best_lanes : cur_lanes);
  } else {
    Totals t;
    TIM_TRY(sample_counts(c, g, model, tim::kModeWidth, seed, phase, 0, sets, 1, nullptr, nullptr, &t));
    nodes = t.nodes;
  }
  static const uint32_t slices[4] = {512, 1024, 2048, 4096};
  const uint32_t cur_slice = c->slice_cap_set;
  uint32_t best_slice = cur_slice;
  double best = 1e300, cur = 1e300;
  for (int i = 0; i < 4; ++i) {
    c->slice_cap = slices[i];
    const double ms = best_ms([&] {
      Totals t;
      return emit_sets(c, g, model, seed, phase, 0, sets, nodes + nodes / 4 + 4096, nullptr, &t);
    });
    if (ms < 0) {
      c->slice_cap = c->slice_cap_set;
      return st;
    }
    r.ms_emit[i] = ms;
    if (slices[i] == cur_slice) cur = ms;
    if (ms < best) {
      best = ms;
      best_slice = slices[i];
    }
  }
  if (!(best < kGain * cur)) best_slice = cur_slice;
  c->slice_cap = c->slice_cap_set = best_slice;
  c->stored.valid = false;
  r.seg_lanes = c->seg_lanes;
  r.slice_cap = best_slice;
  if (out) *out = r;
  return TIM_OK;
}

tim_status tim_spread_mc(tim_ctx* c, const tim_graph* g, int model, uint64_t seed, uint64_t first, uint64_t runs,
                         const int32_t* seeds, int nseeds, uint32_t* d_counts, double* mean, uint64_t* total) {
  TIM_TRY(check_phase_args(c, g, model, 1));
  if (c->serving) return fail(TIM_EINVAL, "a server runs on this context");
  if (nseeds < 0 || (nseeds > 0 && !seeds)) return fail(TIM_EINVAL, "bad seed list");
  for (int i = 0; i < nseeds; ++i)
    if (seeds[i] < 0 || seeds[i] >= g->n) return fail(TIM_EINVAL, "seed %d outside [0, n)", seeds[i]);
  HIP_TRY(hipSetDevice(c->device));
  tim_graph* gm = const_cast<tim_graph*>(g);  // the out-edge lists are a cache of the graph
  TIM_TRY(ensure_out_csr(c, gm));
  TIM_TRY(ensure_big(c, g->n));
  TIM_TRY(ensure(c, c->rr_nodes, (size_t)std::max(nseeds, 1) * 4, "seed list"));
  if (nseeds)
    HIP_TRY(hipMemcpyAsync(c->rr_nodes.p, seeds, (size_t)nseeds * 4, hipMemcpyHostToDevice, c->stream));
  tim::SpreadArgs a;
  memset(&a, 0, sizeof(a));
  a.g.off = g->off;
  a.g.off32 = g->off32;
  a.g.src = g->src;
  a.g.thr = model == TIM_MODEL_IC ? g->thr : nullptr;
  a.g.lthr = model == TIM_MODEL_LT ? g->lthr : nullptr;
  if (model == TIM_MODEL_TRIGGER) {
    a.g.toff = g->toff;
    a.g.tthr = g->tthr;
    a.g.tset = g->tset;
    a.g.tmem = g->tmem;
  }
  a.g.n = g->n;
  a.g.m = g->m;
  a.out_off = gm->out_off;
  a.out_dst = gm->out_dst;
  a.out_eid = gm->out_eid;
  a.seed = seed;
  a.first = first;
  a.runs = runs;
  a.seeds = c->rr_nodes.as<int32_t>();
  a.nseeds = nseeds;
  a.counts = d_counts;
  a.ctr = c->ctr;
  a.stamp = c->big_stamp.as<uint32_t>();
  a.queue = c->big_queue.as<int32_t>();
  a.epoch = c->big_epoch.as<uint32_t>();
  a.stride = (uint64_t)c->big_n;
  a.slots = c->big_slots;
  tim::launch_clear_counters(c->ctr, c->stream);
  if (runs) tim::launch_spread(model, a, c->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(c->ctr_host, c->ctr, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const uint64_t sum = c->ctr_host[1];
  if (total) *total = sum;
  if (mean) *mean = runs ? (double)sum / (double)runs : 0.0;
  return TIM_OK;
}

tim_status tim_run(tim_ctx* c, const tim_graph* g, int model, int k, double eps, double ell, uint64_t seed,
                   uint32_t flags, int32_t* seeds, uint64_t* gains, tim_report* rep) {
  TIM_TRY(check_run_args(c, g, model, k, eps, ell, seeds));
  HIP_TRY(hipSetDevice(c->device));
  return run_impl(c, g, model, k, eps, ell, seed, flags, seeds, gains, rep);
}

tim_status tim_run_batch(tim_ctx* c, tim_query* queries, int count, int max_concurrent, tim_batch_info* info) {
  if (!c || (count > 0 && !queries)) return fail(TIM_EINVAL, "null argument");
  if (count < 0 || max_concurrent < 0) return fail(TIM_EINVAL, "negative count");
  if (c->hub) return fail(TIM_EINVAL, "context is a batch member");
  if (c->serving) return fail(TIM_EINVAL, "a server runs on this context");
  if (info) memset(info, 0, sizeof(*info));
  for (int i = 0; i < count; ++i) {
    tim_query& q = queries[i];
    q.status = check_run_args(c, q.graph, q.model, q.k, q.eps, q.ell, q.seeds);
    if (q.status == TIM_OK && q.model == TIM_MODEL_TRIGGER)
      q.status = fail(TIM_EINVAL, "the general triggering model runs through tim_run, not in batches");
    if (q.status != TIM_OK) return fail(q.status, "query %d: %s", i, g_error.c_str());
  }
  if (count == 0) return TIM_OK;
  HIP_TRY(hipSetDevice(c->device));
  const auto t0 = std::chrono::steady_clock::now();
  const int workers = (max_concurrent == 0 || max_concurrent > count) ? count : max_concurrent;
  if (!c->batch) {
    c->batch = new Hub();
    const tim_status st = hub_setup(c->batch, c);
    if (st != TIM_OK) {
      hub_destroy(c);
      return st;
    }
  }
  Hub& hub = *c->batch;
  int64_t maxn = 2;
  for (int i = 0; i < count; ++i) maxn = std::max<int64_t>(maxn, queries[i].graph->n);
  TIM_TRY(hub_prepare(&hub, c, maxn, workers));
  // Algorithm 2 of every query on the device, then the rest of each query in its worker
  std::vector<tim_kpt_result> kpts;
  TIM_TRY(batch_kpt(c, &hub, queries, count, c->batch_job_cap, &kpts));
  const double ms_kpt = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  std::atomic<int> next{0};
  std::vector<std::string> errs((size_t)count);
  std::thread sched(hub_scheduler, &hub);
  std::vector<std::thread> pool;
  for (int w = 0; w < workers; ++w)
    pool.emplace_back(batch_worker, &hub, c->members[(size_t)w], queries, count, &next, &errs, &kpts);
  for (std::thread& t : pool) t.join();
  {
    std::lock_guard<std::mutex> lk(hub.mu);
    hub.stop = true;
    hub.cv_sched.notify_one();
  }
  sched.join();
  if (info) {
    info->rounds = hub.rounds;
    info->jobs = hub.jobs;
    info->launches = hub.launches;
    info->max_jobs = hub.max_jobs;
    info->workers = (uint64_t)workers;
    info->budget_bytes = hub.limit;
    info->member_budget_bytes = hub.member_budget;
    info->ms_wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    info->ms_kpt = ms_kpt;
    info->kpt_job_cap = c->batch_job_cap;
    info->kpt_steps = hub.kpt_steps;
    info->kpt_graph_launches = hub.kpt_graph_launches;
    info->rr_pool_bytes = hub.rr_total;
    info->rr_peak_bytes = hub.rr_peak;
    info->held_queries = hub.held;
    info->held_ms = hub.held_ms;
  }
  for (int i = 0; i < count; ++i)
    if (queries[i].status != TIM_OK) return fail(queries[i].status, "query %d: %s", i, errs[(size_t)i].c_str());
  return TIM_OK;
}

tim_status tim_autotune_batch(tim_ctx* c, tim_query* queries, int count, tim_batch_tune* out) {
  if (!c || count < 1 || !queries) return fail(TIM_EINVAL, "null argument or no queries");
  if (c->hub) return fail(TIM_EINVAL, "context is a batch member");
  if (c->serving) return fail(TIM_EINVAL, "a server runs on this context");
  for (int i = 0; i < count; ++i) {
    const tim_query& q = queries[i];
    TIM_TRY(check_run_args(c, q.graph, q.model, q.k, q.eps, q.ell, q.seeds));
    if (q.model == TIM_MODEL_TRIGGER)
      return fail(TIM_EINVAL, "the general triggering model runs through tim_run, not in batches");
  }
  HIP_TRY(hipSetDevice(c->device));
  if (!c->batch) {
    c->batch = new Hub();
    const tim_status st = hub_setup(c->batch, c);
    if (st != TIM_OK) {
      hub_destroy(c);
      return st;
    }
  }
  Hub& hub = *c->batch;
  int64_t maxn = 2;
  for (int i = 0; i < count; ++i) maxn = std::max<int64_t>(maxn, queries[i].graph->n);
  TIM_TRY(hub_prepare(&hub, c, maxn, 1));
  tim_batch_tune r;
  memset(&r, 0, sizeof(r));
  const uint64_t caps[4] = {1ull << 16, 1ull << 18, 1ull << 20, 1ull << 22};
  std::vector<tim_kpt_result> kpts;
  int best = -1;
  for (int j = 0; j < 4; ++j) {
    r.caps[j] = caps[j];
    TIM_TRY(batch_kpt(c, &hub, queries, count, caps[j], &kpts));  // untimed
    double t = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
      const auto t0 = std::chrono::steady_clock::now();
      TIM_TRY(batch_kpt(c, &hub, queries, count, caps[j], &kpts));
      t = std::min(t, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    r.ms_kpt[j] = t;
    if (best < 0 || t < r.ms_kpt[best]) best = j;
  }
  // keep the current granularity unless another is 3% faster
  double cur = 1e300;
  for (int j = 0; j < 4; ++j)
    if (caps[j] == c->batch_job_cap) cur = r.ms_kpt[j];
  if (r.ms_kpt[best] < 0.97 * cur) c->batch_job_cap = caps[best];
  r.job_cap = c->batch_job_cap;
  if (out) *out = r;
  return TIM_OK;
}

tim_status tim_server_start(tim_ctx* c, int slots, tim_server** out) {
  if (!c || !out || slots < 1) return fail(TIM_EINVAL, "null argument or slots < 1");
  *out = nullptr;
  if (c->hub) return fail(TIM_EINVAL, "context is a batch member");
  if (c->serving) return fail(TIM_EINVAL, "a server already runs on this context");
  if (c->max_graph_n < 2) return fail(TIM_EINVAL, "upload the graphs before starting a server");
  HIP_TRY(hipSetDevice(c->device));
  if (!c->batch) {
    c->batch = new Hub();
    const tim_status st = hub_setup(c->batch, c);
    if (st != TIM_OK) {
      hub_destroy(c);
      return st;
    }
  }
  TIM_TRY(hub_prepare(c->batch, c, c->max_graph_n, slots));
  c->batch->alive = 0;  // queries in flight, counted as they start and finish
  tim_server* sv = new tim_server();
  sv->ctx = c;
  sv->hub = c->batch;
  sv->slots = slots;
  c->serving = true;
  sv->sched = std::thread(hub_scheduler, sv->hub);
  for (int w = 0; w < slots; ++w) sv->workers.emplace_back(server_worker, sv, c->members[(size_t)w]);
  *out = sv;
  return TIM_OK;
}

tim_status tim_server_submit(tim_server* sv, tim_query* q, uint64_t* ticket) {
  if (!sv || !q || !ticket) return fail(TIM_EINVAL, "null argument");
  tim_ctx* c = sv->ctx;
  TIM_TRY(check_run_args(c, q->graph, q->model, q->k, q->eps, q->ell, q->seeds));
  if (q->model == TIM_MODEL_TRIGGER)
    return fail(TIM_EINVAL, "the general triggering model runs through tim_run, not in servers");
  if ((uint64_t)q->graph->n > sv->hub->big_stride)
    return fail(TIM_EINVAL, "graph uploaded after the server started is larger than its slots");
  Ticket* t = new Ticket();
  t->q = q;
  q->status = TIM_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping) {
      delete t;
      return fail(TIM_EINVAL, "server is stopping");
    }
    t->submitted = std::chrono::steady_clock::now();
    *ticket = (uint64_t)sv->tickets.size();
    sv->tickets.push_back(t);
    sv->queue.push_back(t);
  }
  sv->cv_work.notify_one();
  return TIM_OK;
}

tim_status tim_server_wait(tim_server* sv, uint64_t ticket, double* latency_ms) {
  if (!sv) return fail(TIM_EINVAL, "null server");
  Ticket* t = nullptr;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    if (ticket >= sv->tickets.size()) return fail(TIM_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    t = sv->tickets[(size_t)ticket];
    sv->cv_done.wait(lk, [&] { return t->done; });
  }
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(t->finished - t->submitted).count();
  if (t->q->status != TIM_OK) return fail(t->q->status, "%s", t->err.c_str());
  return TIM_OK;
}

tim_status tim_server_stop(tim_server* sv, tim_batch_info* info) {
  if (!sv) return fail(TIM_EINVAL, "null server");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv_work.notify_all();
  for (std::thread& w : sv->workers) w.join();
  Hub* h = sv->hub;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    h->stop = true;
    h->cv_sched.notify_one();
  }
  sv->sched.join();
  if (info) {
    memset(info, 0, sizeof(*info));
    info->rounds = h->rounds;
    info->jobs = h->jobs;
    info->launches = h->launches;
    info->max_jobs = h->max_jobs;
    info->workers = (uint64_t)sv->slots;
    info->budget_bytes = h->limit;
    info->member_budget_bytes = h->member_budget;
    info->rr_pool_bytes = h->rr_total;
    info->rr_peak_bytes = h->rr_peak;
    info->held_queries = h->held;
    info->held_ms = h->held_ms;
  }
  sv->ctx->serving = false;
  for (Ticket* t : sv->tickets) delete t;
  delete sv;
  return TIM_OK;
}

}  // extern "C"
