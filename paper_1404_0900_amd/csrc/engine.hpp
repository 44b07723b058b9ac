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
  kModeCover = 2   // does R meet a seed set? (Algorithm 3, lines 9-10)
};

// Device counters of one sampling launch (zeroed before it).
enum Counter : int {
  kCtrNextSet = 0,    // next set (relative id) for the wave-level pass
  kCtrDeferred = 1,   // sets handed to the large-set pass
  kCtrPoolCursor = 2, // entries reserved in the node pool
  kCtrNextBig = 3,    // next deferred set for the large-set pass
  kCtrKappaLo = 4,    // exact sum of kappa * 2^53 (128 bits)
  kCtrKappaHi = 5,
  kCtrWidth = 6,      // sum of w(R)
  kCtrNodes = 7,      // sum of |R|
  kCtrCovered = 8,    // sets meeting the seed set
  kCtrCount = 16
};

struct GraphView {
  const int64_t* off;   // n+1
  const int32_t* src;   // m rounded up to a multiple of 4, plus 4, zero padded
  const uint32_t* thr;  // same padding, or nullptr for the weighted cascade
  int64_t n, m;
};

struct SampleArgs {
  GraphView g;
  uint64_t seed;
  uint32_t phase;
  uint64_t first, count;
  int k;                          // kappa exponent (width mode)
  unsigned long long* ctr;        // kCtrCount counters
  uint64_t* widths;               // per set, nullable
  uint32_t* sizes;                // per set, nullable
  int32_t* pool;                  // emit: node pool
  uint64_t pool_cap;
  uint64_t* set_start;            // emit: pool offset of each set
  uint32_t* set_len;              // emit: size of each set
  const uint32_t* seed_bits;      // cover: n-bit membership of the seed set
  uint64_t* deferred;             // relative ids of sets for the large-set pass
  uint64_t deferred_cap;
  // large-set pass: per-slot visited stamps and queues (n entries each)
  uint32_t* big_stamp;
  int32_t* big_queue;
  uint32_t* big_epoch;
  int big_slots;
};

// ---- sample.hip ----
void launch_clear_counters(unsigned long long* ctr, hipStream_t s);
int ic_wave_blocks_per_cu(int mode, bool wc);
int lt_lane_blocks_per_cu(int mode);
void launch_sample(int model, int mode, const SampleArgs& a, int grid_small, hipStream_t s);
void launch_sample_large(int model, int mode, const SampleArgs& a, hipStream_t s);

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
  const int64_t* set_off;
  const int32_t* nodes;
  uint32_t* cnt;       // n: coverage counts
  uint32_t* fill;      // n: scatter cursors
  int64_t* inv_off;    // n+1
  uint32_t* inv_sets;  // total entries
  uint8_t* covered;    // nsets
  uint8_t* selected;   // n
  unsigned long long* best;  // k packed (count, ~id) keys
  void* scan_temp;
};
void launch_index(const GreedyArgs& a, hipStream_t s);
void launch_greedy(const GreedyArgs& a, int k, hipStream_t s);

}  // namespace tim
