// Internal interface between the host driver (api.cpp) and the kernels
// (sample.hip, coverage.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tim {

// What a sampling launch does with each RR set.
enum SampleMode : int {
  kModeWidth = 0,  // w(R), |R| and kappa(R) only (Algorithm 2)
  kModeEmit = 1,   // store the nodes of R (Algorithms 1 and 3)
  kModeCover = 2   // does R meet a seed set? (Algorithm 3, RefineKPT's test)
};

// Device counters of one sampling launch (zeroed before it).  Sets flow
// through up to three tiers: tier 0 takes the launch's range of set ids and
// hands sets that outgrow its on-chip structures to list 1; tier 1 (IC only)
// takes list 1 and hands the rest to list 2; the last tier finishes list 2
// (IC: device-memory visited stamps) or list 1 (LT: the stamp-free chain
// tier).  Each tier has its own block of accumulators at kCtrAcc +
// kAccStride * tier.  The cursors and list lengths, which every wavefront
// updates with device atomics, sit in 128-byte lines of their own: atomics on
// different words of one line wait for each other (a 4M-set stored-set launch
// took 6% longer with them packed into one line).  The first two tiers of the
// single-job launches (IC, triggering; the LT lane tier) split their range
// into kCtrParts parts, each with a cursor of its own: block b starts on part
// b mod kCtrParts (blocks take turns over the XCDs) and moves on to the next
// part when its part is spent, so that the wavefronts' refills meet on eight
// cursors instead of one (with one, a TIM+ step on the 1M-node graph took 5%
// longer under IC and 18% longer under LT).
enum Counter : int {
  kCtrParts = 8,         // cursors of tiers 0 and 1: one per part of their range
  kCtrPartStride = 16,   // words between them
  kCtrNext0 = 0,         // tier-0 cursors over the range (kCtrParts of them)
  kCtrList1 = 128,       // length of list 1
  kCtrNext1 = 144,       // tier-1 cursors over list 1 (kCtrParts of them)
  kCtrList2 = 272,       // length of list 2
  kCtrNext2 = 288,       // last-tier cursor
  kCtrPoolCursor = 304,  // node-pool entries reserved
  kCtrAcc = 320,
  kAccKappaLo = 0,     // exact sum of kappa * 2^53 (128 bits)
  kAccKappaHi = 1,
  kAccWidth = 2,       // sum of w(R): edges examined
  kAccNodes = 3,       // sum of |R| (coverage mode: nodes reached before the first seed)
  kAccCovered = 4,     // sets meeting the seed set
  kAccStride = 8,
  kCtrCount = kCtrAcc + 3 * kAccStride
};

// Where one tier reads its sets and where it sends the ones it defers.
struct TierIO {
  const uint64_t* in_list;  // relative set ids, or nullptr for the range [0, count)
  int in_len_ctr;           // counter holding the length of in_list
  int next_ctr;             // work cursor
  uint64_t* out_list;       // deferred sets (relative ids), capacity = count
  int out_len_ctr;
  int acc;                  // accumulator block (tier number)
  int parts;                // 0 or 1: one cursor at next_ctr; else `parts` cursors kCtrPartStride apart, one per part
};

// Node-pool entries a wavefront reserves at a time when it stores sets (the
// default; SampleArgs::pool_chunk sets it per launch).
constexpr uint32_t kPoolChunk = 2048;

struct GraphView {
  const int64_t* off;   // n+1
  const uint32_t* off32;  // the same offsets in 32 bits (m < 2^32), for the IC first tiers
  const int32_t* src;   // m rounded up to a multiple of 4, plus 4, zero padded
  const uint32_t* thr;  // same padding, or nullptr for the weighted cascade
  const uint32_t* lthr; // LT cumulative in-weight thresholds (m), or nullptr for 1/indeg
  // general triggering model: outcomes of v are [toff[v], toff[v+1]) with
  // cumulative thresholds tthr; outcome j's members (local in-edge indices)
  // are tmem[tset[j] .. tset[j+1])
  const int64_t* toff;
  const uint32_t* tthr;
  const int64_t* tset;
  const uint32_t* tmem;
  int64_t n, m;
};

struct SampleArgs {
  GraphView g;
  uint64_t seed;
  uint32_t phase;
  uint64_t first, count;
  int k;                          // kappa exponent (width mode)
  unsigned long long* ctr;        // kCtrCount counters
  uint64_t* widths;               // per set, nullable (store mode; width mode: copied from wbuf)
  uint32_t* sizes;                // per set, nullable
  uint32_t* wbuf;                 // width mode: w(R) of every set of the launch
  int32_t* pool;                  // emit: this launch's part of the node pool
  uint64_t pool_cap;              // entries in it
  uint64_t pool_base;             // its offset in the whole pool (added to set_start)
  uint32_t pool_chunk;            // entries a wavefront reserves at a time (>= 1)
  uint64_t* set_start;            // emit: pool offset of each set
  uint32_t* set_len;              // emit: size of each set
  const uint32_t* seed_bits;      // cover: n-bit membership of the seed set
  uint64_t* list1;                // deferred lists (capacity count each)
  uint64_t* list2;
  // last tier: per-slot visited stamps and queues (n entries each)
  uint32_t* big_stamp;
  int32_t* big_queue;
  uint32_t* big_epoch;
  int big_slots;
  uint64_t big_stride;  // entries per slot in big_stamp / big_queue (>= n)
};

// ---- sample.hip ----
void launch_clear_counters(unsigned long long* ctr, hipStream_t s);
// Lanes per set of the IC tier-0 kernel: 4, 8, 16, 32 or 64 (environment
// variable TIM_IC_SEG_LANES, read when a context is created; default 8).
int ic_seg_lanes();
int ic_blocks_per_cu(int mode, bool wc, int seg_lanes);
int ic_tier1_blocks_per_cu(int mode, bool wc);
int lt_lane_blocks_per_cu(int mode);
// Occupancy of the general-triggering first tier (one set per wavefront).
int trig_blocks_per_cu(int mode);         // tier 0 of the triggering model
int trig_tier1_blocks_per_cu(int mode);   // its one-set-per-wavefront tier
// Occupancy of the LT long-chain tier (single or batched launches).
int lt_chain_blocks_per_cu(int mode, bool batch);
// Largest set the first tier keeps in LDS (IC: its queue for seg_lanes lanes
// per set; LT: its chain); larger sets go on to the next tier.
uint32_t tier0_set_cap(int model, int seg_lanes);
// Tier 0 (grid0 blocks; IC with seg_lanes lanes per set), then the deferral
// tiers (grid1 blocks: IC tier 1, or the LT long-chain tier).  after_tier0,
// if given, is recorded between tier 0 and the rest.
void launch_sample(int model, int mode, const SampleArgs& a, int seg_lanes, int grid0, int grid1, hipStream_t s,
                   hipEvent_t after_tier0);

// Sampling jobs of several queries in one launch (device array of njobs
// SampleArgs, 1 <= njobs <= 64, one mode and model; all jobs point at the
// same last-tier slots).  Tier 0 of IC uses 8 lanes per set.
struct JobTable {
  const SampleArgs* jobs;
  int njobs;
  int spread;  // 1: wavefronts start spread over the jobs in proportion to their sets (jobs of one graph)
};
constexpr int kMaxBatchJobs = 64;
// Occupancy of the batched tier-0 (tier 0) or tier-1 (tier 1, IC) kernel.
int batch_blocks_per_cu(int model, int mode, bool wc, int tier);
void launch_clear_counters_batch(const JobTable& t, hipStream_t s);
// All tiers and the kappa sums; max_count is the largest job's count.  grid1
// is the IC tier-1 or LT long-chain grid, slots the IC last-tier slots.
// after_tier0, if given, is recorded between tier 0 and the rest.
void launch_sample_batch(int model, int mode, bool wc, const JobTable& t, int grid0, int grid1, int slots,
                         uint64_t max_count, hipStream_t s, hipEvent_t after_tier0);

// ---- device-driven KptEstimation for a batch of queries (sample.hip) ----
// Algorithm 2 for up to kMaxBatchJobs queries of one (model, thresholds)
// class, with the round loop on the device: each step hands every query a
// chunk of its current round (a device work queue of set-id ranges, at most
// job_cap sets per query and step_cap in all), runs the batched samplers on
// those chunks, and adds each chunk's totals to its round; a round whose sets
// are all done takes the stop test S * 2^i > c_i * 2^53 and the query moves
// to round i + 1 or stops.  The steps need no host synchronisation, so a
// run of them is captured in one HIP graph.
constexpr int kKptMaxRounds = 64;
struct KptQuery {
  GraphView g;
  uint64_t seed;
  int32_t k, imax;
  int32_t round;  // current round (1-based); 0 once stopped
  int32_t i_last;  // round that stopped (imax if none did)
  int32_t err;     // a deferred-set list overflowed
  int32_t pad;
  uint64_t pos;    // next set id of the current round
  unsigned long long sum_lo, sum_hi, width, nodes;  // totals of the current round so far
  uint64_t c[kKptMaxRounds];
  unsigned long long r_lo[kKptMaxRounds], r_hi[kKptMaxRounds], r_width[kKptMaxRounds], r_nodes[kKptMaxRounds];
};
struct KptStepArgs {
  KptQuery* q;
  int nq;
  SampleArgs* jobs;            // nq job descriptors (rewritten every step)
  unsigned long long* ctr;     // nq * kCtrCount counters
  uint32_t* wbuf;              // step_cap widths
  uint64_t* list1;             // step_cap deferred ids
  uint64_t* list2;             // step_cap deferred ids (IC)
  uint64_t step_cap, job_cap;  // sets per step in all / per query
  unsigned int* active;        // queries not yet stopped after the last step
  uint32_t* big_stamp;
  int32_t* big_queue;
  uint32_t* big_epoch;
  int big_slots;
  uint64_t big_stride;
};
void launch_kpt_jobs(const KptStepArgs& a, hipStream_t s);
void launch_kpt_advance(const KptStepArgs& a, hipStream_t s);

// ---- spread.hip ----
// Forward Monte-Carlo runs [first, first+runs) of phase 65 from a seed set.
struct SpreadArgs {
  GraphView g;                // in-CSR (coins, thresholds, LT picks)
  const int64_t* out_off;     // n+1
  const int32_t* out_dst;     // m: head of each out-edge
  const uint32_t* out_eid;    // m: its in-CSR edge id
  uint64_t seed, first, runs;
  const int32_t* seeds;       // nseeds node ids (repeats allowed)
  int nseeds;
  uint32_t* counts;           // per run, nullable
  unsigned long long* ctr;    // [0] run cursor, [1] sum of the runs' spreads (cleared by the caller)
  uint32_t* stamp;            // per slot: n stamps and an n-entry queue, stride entries apart
  int32_t* queue;
  uint32_t* epoch;
  uint64_t stride;
  int slots;
};
void launch_out_csr_count(const int32_t* src, int64_t m, uint32_t* cnt, hipStream_t s);
void launch_out_csr_scatter(const int64_t* in_off, const int32_t* src, int64_t n, int64_t m, const int64_t* out_off,
                            uint32_t* fill, int32_t* out_dst, uint32_t* out_eid, hipStream_t s);
void launch_spread(int model, const SpreadArgs& a, hipStream_t s);

// ---- coverage.hip ----
// out[0..len] = exclusive prefix sums of in[0..len), out[len] = total.
size_t scan_temp_bytes(uint64_t len);
void launch_scan_u32_to_i64(const uint32_t* in, int64_t* out, uint64_t len, void* temp, hipStream_t s);
void launch_compact(const int32_t* pool, const uint64_t* set_start, const uint32_t* set_len, const int64_t* out_off,
                    int32_t* out_nodes, uint64_t nsets, hipStream_t s);
void launch_check_ids(const int32_t* nodes, uint64_t total, int64_t n, unsigned int* flag, hipStream_t s);
void launch_set_sizes(const int64_t* set_off, uint32_t* sizes, uint64_t nsets, hipStream_t s);
// Inverted index of a CSR collection and the greedy maximum coverage.
struct GreedyArgs {
  int64_t n;
  uint64_t nsets;
  uint64_t total;      // entries of the collection
  // layout: CSR (set_off, n+1 offsets into nodes) if set_off is set, else the
  // node pool of an emit launch (set s: set_len[s] nodes from nodes[set_start[s]])
  const int64_t* set_off;
  const uint64_t* set_start;
  const uint32_t* set_len;
  const int32_t* nodes;
  uint32_t* cnt;       // n: coverage counts
  uint32_t* fill;      // n: scatter cursors
  int64_t* inv_off;    // n+1
  uint32_t* inv_sets;  // total entries
  uint8_t* covered;    // nsets
  uint8_t* selected;   // n
  unsigned long long* best;  // k packed (count, ~id) keys
  void* scan_temp;
  void* bkt;           // optional: bucket_workspace_bytes(n, total, index) for the counting sort by node range
};
// Workspace of the counting sort by node range that launch_counts and
// launch_index use when GreedyArgs.bkt is set; 0 where it does not apply.
size_t bucket_workspace_bytes(int64_t n, uint64_t total, bool index);
// Coverage counts only (the greedy of k = 1 needs no index).
void launch_counts(const GreedyArgs& a, hipStream_t s);
void launch_index(const GreedyArgs& a, hipStream_t s);
void launch_greedy(const GreedyArgs& a, int k, hipStream_t s);
// The same greedy one step at a time, for collections of which only sets
// [0, a.nsets) are stored (the rest is regenerated in parts between steps):
// init clears covered[0, covered_len), the selections and the k keys;
// argmax writes key j and marks the chosen node selected; cover takes the
// stored sets containing it out of the counts.
void launch_zero_counts(uint32_t* cnt, int64_t n, hipStream_t s);
void launch_greedy_init(const GreedyArgs& a, uint64_t covered_len, int k, hipStream_t s);
void launch_argmax_step(const GreedyArgs& a, int j, hipStream_t s);
void launch_cover_step(const GreedyArgs& a, int j, hipStream_t s);
// Sets left in the node pool by an emit launch (set j: set_len[j] nodes from
// pool[set_start[j]]).  pool_hist adds their memberships to cnt; pool_cover
// marks those not yet covered that contain the node of key *best (covered
// indexed like the sets) and takes them out of the counts of their members.
void launch_pool_hist(const int32_t* pool, const uint64_t* set_start, const uint32_t* set_len, uint64_t nsets,
                      uint32_t* cnt, hipStream_t s);
void launch_pool_cover(const unsigned long long* best, const int32_t* pool, const uint64_t* set_start,
                       const uint32_t* set_len, uint64_t nsets, uint8_t* covered, uint32_t* cnt, hipStream_t s);

// The greedy's work arrays in one fixed device array (for callers that cannot
// allocate): limits, the per-device lookup of its address (call once per
// device with that device current), and the layout of the arrays in it.
constexpr int64_t kStaticMaxN = 1 << 20;          // nodes
constexpr uint64_t kStaticMaxSets = 1ull << 22;   // sets of the collection
constexpr uint64_t kStaticMaxEntries = 1ull << 23;  // total size of the collection
constexpr int kStaticMaxK = 1024;                 // greedy steps
constexpr int kStaticMaxDevices = 64;
struct StaticGreedy {
  uint32_t* cnt;
  uint32_t* fill;
  int64_t* inv_off;
  uint32_t* inv_sets;
  uint8_t* covered;
  uint8_t* selected;
  unsigned long long* best;
  unsigned int* flag;  // id check
  int64_t* zero_off;   // CSR offset of an empty collection
  void* scan_temp;
};
size_t static_scratch_bytes();
hipError_t static_scratch_init(int device);
// All pointers null if static_scratch_init has not succeeded on the device.
StaticGreedy static_greedy_layout(int device);
void launch_set_u64(unsigned long long* p, unsigned long long v, hipStream_t s);

}  // namespace tim
