// RR collection layout and greedy maximum coverage on gfx950.
//
// Compaction (scan of set sizes, then a gather) turns the node pool written by
// the samplers into a flat CSR of sets in set-id order.  A counting sort of
// that CSR (histogram, scan, scatter) builds the node -> sets inverted index;
// its histogram is also the initial coverage count of every node.  The greedy
// of Algorithm 1 then runs on the device without host round
// trips: per step one argmax kernel packs (count, ~id) into a 64-bit key so
// that a single atomicMax selects the largest count with ties to the lowest
// id, and one cover kernel marks the chosen node's uncovered sets and
// decrements the counts of their members.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "engine.hpp"

namespace tim {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long x, unsigned long long* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  if (lane == 0) red[wv] = x;
  __syncthreads();
  unsigned long long t = 0;
  for (int w = 0; w < kThreads / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Exclusive block scan of 64-bit values (256 threads).
__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long x, unsigned long long* red,
                                                              unsigned long long* total) {
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  unsigned long long incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) red[wv] = incl;
  __syncthreads();
  unsigned long long carry = 0, all = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wv) carry += red[w];
    all += red[w];
  }
  __syncthreads();
  *total = all;
  return carry + incl - x;
}

__global__ __launch_bounds__(kThreads) void scan_tile_sums(const uint32_t* in, uint64_t len,
                                                           unsigned long long* tile_sums) {
  __shared__ unsigned long long red[kThreads / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  unsigned long long s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint64_t j = base + (uint64_t)i * kThreads + threadIdx.x;
    if (j < len) s += in[j];
  }
  s = block_sum_u64(s, red);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void scan_tile_offsets(unsigned long long* tile_sums, uint64_t ntiles,
                                                              int64_t* out, uint64_t len) {
  __shared__ unsigned long long red[kThreads / 64];
  unsigned long long carry = 0;
  for (uint64_t base = 0; base < ntiles; base += kThreads) {
    const uint64_t j = base + threadIdx.x;
    const unsigned long long x = j < ntiles ? tile_sums[j] : 0ull;
    unsigned long long total;
    const unsigned long long ex = block_excl_scan(x, red, &total);
    if (j < ntiles) tile_sums[j] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) out[len] = (int64_t)carry;
}

__global__ __launch_bounds__(kThreads) void scan_apply(const uint32_t* in, uint64_t len,
                                                       const unsigned long long* tile_off, int64_t* out) {
  __shared__ unsigned long long red[kThreads / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kItems;
  uint32_t v[kItems];
  unsigned long long s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    v[i] = (base + i < len) ? in[base + i] : 0u;
    s += v[i];
  }
  unsigned long long total;
  unsigned long long run = tile_off[blockIdx.x] + block_excl_scan(s, red, &total);
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    if (base + i < len) out[base + i] = (int64_t)run;
    run += v[i];
  }
}

__global__ void compact_kernel(const int32_t* pool, const uint64_t* set_start, const uint32_t* set_len,
                               const int64_t* out_off, int32_t* out_nodes, uint64_t nsets) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nsets; s += stride) {
    const int32_t* from = pool + set_start[s];
    int32_t* to = out_nodes + out_off[s];
    const uint32_t len = set_len[s];
    for (uint32_t i = 0; i < len; ++i) to[i] = from[i];
  }
}

// flag[0] |= 1 if any node id of the collection lies outside [0, n).
__global__ void check_ids_kernel(const int32_t* nodes, uint64_t total, int64_t n, unsigned int* flag) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
    bad |= nodes[i] < 0 || (int64_t)nodes[i] >= n;
  if (bad) atomicOr(flag, 1u);
}

__global__ void set_sizes_kernel(const int64_t* set_off, uint32_t* sizes, uint64_t nsets) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nsets; s += stride)
    sizes[s] = (uint32_t)(set_off[s + 1] - set_off[s]);
}

// Counters that many blocks update with device atomics sit one per 128-byte
// line (32 words apart): atomics on different words of one line wait for each
// other.  The counting sort's per-bucket counts and cursors took 0.45 ms more
// per TIM+ step on the 1M-node graph packed 32 to a line.
constexpr int kLinePad = 32;

__global__ void unpad_u32(const uint32_t* in, uint32_t* out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[(size_t)i * kLinePad];
}

__global__ void zero_u32(uint32_t* p, uint64_t len) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = 0u;
}

__global__ void zero_u8(uint8_t* p, uint64_t len) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = 0u;
}

__global__ void zero_u64(unsigned long long* p, uint64_t len) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) p[i] = 0ull;
}

// ---- views of a collection: set s has len(s) nodes from nodes[start(s)] ----
struct CsrSets {  // flat CSR (caller collections, resident prefixes)
  const int64_t* off;
  const int32_t* nodes;
  __device__ __forceinline__ int64_t start(uint64_t s) const { return off[s]; }
  __device__ __forceinline__ uint32_t len(uint64_t s) const { return (uint32_t)(off[s + 1] - off[s]); }
};
struct PoolSets {  // node pool as the samplers leave it (per-set start and size)
  const uint64_t* st;
  const uint32_t* ln;
  const int32_t* nodes;
  __device__ __forceinline__ int64_t start(uint64_t s) const { return (int64_t)st[s]; }
  __device__ __forceinline__ uint32_t len(uint64_t s) const { return ln[s]; }
};

// ---- per-tile aggregation of node updates in LDS ----
// A tile's updates to the same node (hub nodes recur in many RR sets) are
// summed in an LDS open-addressing table (at most about half full for a tile
// of typical sets) and reach device memory as one atomic per distinct node
// per tile.  A node that finds no free slot among the first kAggProbes of its
// probe sequence falls back to direct atomics: a tile holding a set larger
// than the table (a set reaching a giant component) fills it, and without
// the bound every later entry would scan the whole table.  Probe sequences
// are fixed per node and slots are never freed within a tile, so a node is
// either in the table for all of its entries of the tile or for none.
constexpr int kAggLog = 12;
constexpr int kAgg = 1 << kAggLog;
constexpr int kAggProbes = 32;
constexpr int kTileSets = 128;      // sets per tile (set-tiled kernels)
constexpr int kHistTileSets = 256;  // sets per tile of the counts pass (at most kThreads)
static_assert(kTileSets <= kThreads && kHistTileSets <= kThreads, "a tile's sets are carried one per thread");
constexpr int kTileEntries = 2048;  // entries per tile (flat histogram)

// lg: the table's size in use, 2^lg <= kAgg slots.
__device__ __forceinline__ int agg_slot(uint32_t* keys, uint32_t u, bool insert, int lg = kAggLog) {
  const uint32_t key = u + 1u;
  const uint32_t mask = (1u << lg) - 1u;
  uint32_t pos = (u * 0x9E3779B1u) >> (32 - lg);
  for (int i = 0; i < kAggProbes; ++i) {
    const uint32_t cur = keys[pos];
    if (cur == key) return (int)pos;
    if (cur == 0u) {
      if (!insert) return -1;
      const uint32_t old = atomicCAS(&keys[pos], 0u, key);
      if (old == 0u || old == key) return (int)pos;
    }
    pos = (pos + 1u) & mask;
  }
  return -1;
}

// Clears the first `slots` (a multiple of 4) slots of a table.
__device__ __forceinline__ void agg_clear(uint32_t* a, uint32_t* b, int slots = kAgg) {
  uint4* a4 = reinterpret_cast<uint4*>(a);
  uint4* b4 = reinterpret_cast<uint4*>(b);
  for (int i = threadIdx.x; i < slots / 4; i += blockDim.x) {
    a4[i] = make_uint4(0u, 0u, 0u, 0u);
    if (b) b4[i] = make_uint4(0u, 0u, 0u, 0u);
  }
}

// Block-wide prefix of the sizes of a tile's sets: thread t < kTileSets
// carries set t (len 0 if it takes no part); afterwards s_pre[t] is the first
// tile position of set t, s_pre[kTileSets] the tile total, and s_start[t] its
// first entry in the collection.
template <int TS = kTileSets>
__device__ __forceinline__ void tile_prefix(uint32_t len, int64_t start, int64_t* s_start, int64_t* s_pre,
                                            uint32_t* s_wtot) {
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  uint32_t incl = len;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_wtot[wv] = incl;
  __syncthreads();
  uint32_t carry = 0;
  for (int w = 0; w < wv; ++w) carry += s_wtot[w];
  if (threadIdx.x < TS) {
    s_start[threadIdx.x] = start;
    s_pre[threadIdx.x + 1] = carry + incl;
  }
  if (threadIdx.x == 0) s_pre[0] = 0;
  __syncthreads();
}

// Position of tile entry e among the tile's sets: the set j with
// s_pre[j] <= e < s_pre[j+1].
__device__ __forceinline__ int tile_set_of(const int64_t* s_pre, int ns, int64_t e) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_pre[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int TS = kTileSets>
struct TileShared {
  int64_t start[TS];
  int64_t pre[TS + 1];
  uint32_t wtot[kThreads / 64];
  uint32_t key[kAgg], cnt[kAgg];
};

// Tiles without entries (a greedy step's cover pass mostly meets tiles whose
// sets are all covered already) skip the LDS table altogether.  Smaller
// tiles still aggregate: the nodes they share are hubs, whose direct atomics
// would contend across the chip.
constexpr int64_t kAggMin = 1;

// Adds (sign +1) or subtracts the memberships of the tile's listed sets (prefix
// from tile_prefix) to cnt, skipping node `skip`.
// The table in use for a tile of `tot` entries: at least twice as many slots
// as entries (256 to kAgg), so that a tile of few entries, as most tiles of
// the cover pass are, clears and scans few slots.
__device__ __forceinline__ int agg_log_for(int64_t tot) {
  int lg = 8;
  while (lg < kAggLog && (int64_t(1) << lg) < 2 * tot) ++lg;
  return lg;
}

template <bool kAdd, int TS = kTileSets>
__device__ __forceinline__ void tile_apply(const int32_t* nodes, TileShared<TS>& t, int64_t skip, uint32_t* cnt) {
  const int64_t tot = t.pre[TS];
  const bool agg = tot >= kAggMin;
  const int lg = agg_log_for(tot);
  if (agg) {
    agg_clear(t.key, t.cnt, 1 << lg);
    __syncthreads();
  }
  for (int64_t e = threadIdx.x; e < tot; e += kThreads) {
    const int j = tile_set_of(t.pre, TS, e);
    const int32_t u = nodes[t.start[j] + (e - t.pre[j])];
    if (u == skip) continue;
    const int slot = agg ? agg_slot(t.key, (uint32_t)u, true, lg) : -1;
    if (slot >= 0) atomicAdd(&t.cnt[slot], 1u);
    else if (kAdd) atomicAdd(&cnt[u], 1u);
    else atomicSub(&cnt[u], 1u);
  }
  if (agg) {
    __syncthreads();
    for (int i = threadIdx.x; i < (1 << lg); i += kThreads) {
      if (t.key[i]) {
        if (kAdd) atomicAdd(&cnt[t.key[i] - 1u], t.cnt[i]);
        else atomicSub(&cnt[t.key[i] - 1u], t.cnt[i]);
      }
    }
  }
  __syncthreads();
}

// cnt[u] += number of sets containing u, over a flat entry array.
__global__ __launch_bounds__(kThreads) void hist_flat_kernel(const int32_t* nodes, uint64_t total, uint32_t* cnt) {
  __shared__ uint32_t s_key[kAgg], s_cnt[kAgg];
  for (uint64_t t0 = (uint64_t)blockIdx.x * kTileEntries; t0 < total; t0 += (uint64_t)gridDim.x * kTileEntries) {
    agg_clear(s_key, s_cnt);
    __syncthreads();
    const uint64_t t1 = min(t0 + (uint64_t)kTileEntries, total);
    for (uint64_t e = t0 + threadIdx.x; e < t1; e += kThreads) {
      const uint32_t u = (uint32_t)nodes[e];
      const int slot = agg_slot(s_key, u, true);
      if (slot >= 0) atomicAdd(&s_cnt[slot], 1u);
      else atomicAdd(&cnt[u], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kAgg; i += kThreads)
      if (s_key[i]) atomicAdd(&cnt[s_key[i] - 1u], s_cnt[i]);
    __syncthreads();
  }
}

// cnt[u] += number of sets containing u, in tiles of sets.
// (Larger tiles than the other passes: the LDS table's clear and scan are
// spread over twice the entries, and more hub repeats meet in it.)
template <class V>
__global__ __launch_bounds__(kThreads) void hist_sets_kernel(V sets, uint64_t nsets, uint32_t* cnt) {
  constexpr int TS = kHistTileSets;
  __shared__ TileShared<TS> t;
  for (uint64_t s0 = (uint64_t)blockIdx.x * TS; s0 < nsets; s0 += (uint64_t)gridDim.x * TS) {
    const int ns = (int)min((uint64_t)TS, nsets - s0);
    uint32_t len = 0;
    int64_t start = 0;
    if (threadIdx.x < ns) {
      start = sets.start(s0 + threadIdx.x);
      len = sets.len(s0 + threadIdx.x);
    }
    tile_prefix<TS>(len, start, t.start, t.pre, t.wtot);
    tile_apply<true, TS>(sets.nodes, t, -1, cnt);
  }
}

// inv_sets[inv_off[u] ..] = the sets containing u, in no particular order.
template <class V>
__global__ __launch_bounds__(kThreads) void scatter_kernel(V sets, uint64_t nsets, const int64_t* inv_off,
                                                           uint32_t* fill, uint32_t* inv_sets) {
  __shared__ TileShared<> t;
  __shared__ uint32_t s_base[kAgg];
  for (uint64_t s0 = (uint64_t)blockIdx.x * kTileSets; s0 < nsets; s0 += (uint64_t)gridDim.x * kTileSets) {
    const int ns = (int)min((uint64_t)kTileSets, nsets - s0);
    agg_clear(t.key, t.cnt);
    uint32_t len = 0;
    int64_t start = 0;
    if (threadIdx.x < ns) {
      start = sets.start(s0 + threadIdx.x);
      len = sets.len(s0 + threadIdx.x);
    }
    tile_prefix(len, start, t.start, t.pre, t.wtot);
    const int64_t tot = t.pre[kTileSets];
    for (int64_t e = threadIdx.x; e < tot; e += kThreads) {
      const int j = tile_set_of(t.pre, kTileSets, e);
      const int slot = agg_slot(t.key, (uint32_t)sets.nodes[t.start[j] + (e - t.pre[j])], true);
      if (slot >= 0) atomicAdd(&t.cnt[slot], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kAgg; i += kThreads) {
      if (t.key[i]) s_base[i] = atomicAdd(&fill[t.key[i] - 1u], t.cnt[i]);
      t.cnt[i] = 0u;
    }
    __syncthreads();
    for (int64_t e = threadIdx.x; e < tot; e += kThreads) {
      const int j = tile_set_of(t.pre, kTileSets, e);
      const uint32_t u = (uint32_t)sets.nodes[t.start[j] + (e - t.pre[j])];
      const uint32_t sid = (uint32_t)(s0 + (uint64_t)j);
      const int slot = agg_slot(t.key, u, false);
      uint64_t pos;
      if (slot >= 0) pos = (uint64_t)inv_off[u] + s_base[slot] + atomicAdd(&t.cnt[slot], 1u);
      else pos = (uint64_t)inv_off[u] + atomicAdd(&fill[u], 1u);
      inv_sets[pos] = sid;
    }
    __syncthreads();
  }
}

// ---- counting sort of the entries by node range ----
//
// The counts pass above adds one device atomic per distinct node of every
// tile, about two for every three entries on the large collections, and
// device atomics to scattered addresses top out far below the memory's
// bandwidth.  With a workspace, the index is built instead by a counting sort
// in two levels: the entries are first moved into buckets of 2^shift
// consecutive node ids (one atomic per bucket and tile of sets), then each
// chunk of a bucket counts its nodes, and places its sets, in LDS, with one
// device atomic per distinct node and chunk (none for a bucket of one chunk).
// Counts and index are those of the direct passes: only the order of the sets
// within a node's list differs, and no step of the greedy depends on it.
// Buckets of 8192 nodes (32 KB of LDS counters per chunk): the fewer the
// buckets, the longer the runs each tile of sets writes into one bucket.
// Chunks of 16384 entries give the per-bucket passes four times the blocks of
// 65536-entry chunks, for one more atomic per node present in each extra chunk:
// the index and greedy run about 7% faster on a 1M-node graph.
constexpr int kBucketShiftMin = 13, kBucketShiftMax = 13;
constexpr int kBucketMax = 8192;             // buckets (LDS counters per tile of sets)
constexpr uint32_t kBucketChunk = 1u << 14;  // entries per block of the per-bucket passes

// bcnt[b * kLinePad] += entries of the collection in bucket b.
template <class V>
__global__ __launch_bounds__(kThreads) void bucket_hist_kernel(V sets, uint64_t nsets, int shift, int nb,
                                                               uint32_t* bcnt) {
  constexpr int TS = kHistTileSets;
  __shared__ int64_t s_start[TS];
  __shared__ int64_t s_pre[TS + 1];
  __shared__ uint32_t s_wtot[kThreads / 64];
  __shared__ uint32_t h[kBucketMax];
  for (uint64_t s0 = (uint64_t)blockIdx.x * TS; s0 < nsets; s0 += (uint64_t)gridDim.x * TS) {
    uint32_t len = 0;
    int64_t start = 0;
    if (threadIdx.x < TS && s0 + threadIdx.x < nsets) {
      start = sets.start(s0 + threadIdx.x);
      len = sets.len(s0 + threadIdx.x);
    }
    for (int i = threadIdx.x; i < nb; i += kThreads) h[i] = 0u;
    tile_prefix<TS>(len, start, s_start, s_pre, s_wtot);
    const int64_t tot = s_pre[TS];
    for (int64_t e = threadIdx.x; e < tot; e += kThreads) {
      const int j = tile_set_of(s_pre, TS, e);
      const uint32_t u = (uint32_t)sets.nodes[s_start[j] + (e - s_pre[j])];
      atomicAdd(&h[u >> shift], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += kThreads)
      if (h[i]) atomicAdd(&bcnt[(size_t)i * kLinePad], h[i]);
    __syncthreads();
  }
}

// Chunks of kBucketChunk entries per bucket: cstart[b] is bucket b's first
// chunk, cstart[nb] their number, cb[c] the bucket of chunk c.
__global__ __launch_bounds__(kThreads) void bucket_chunks_kernel(const int64_t* boff, int nb, uint32_t* cstart,
                                                                 uint32_t* cb) {
  __shared__ unsigned long long red[kThreads / 64];
  unsigned long long carry = 0;
  for (int base = 0; base < nb; base += kThreads) {
    const int b = base + (int)threadIdx.x;
    const unsigned long long len = b < nb ? (unsigned long long)(boff[b + 1] - boff[b]) : 0ull;
    const unsigned long long ch = (len + kBucketChunk - 1) / kBucketChunk;
    unsigned long long total;
    const unsigned long long ex = block_excl_scan(ch, red, &total);
    if (b < nb) {
      const uint32_t c0 = (uint32_t)(carry + ex);
      cstart[b] = c0;
      for (uint32_t j = 0; j < (uint32_t)ch; ++j) cb[c0 + j] = (uint32_t)b;
    }
    carry += total;
  }
  if (threadIdx.x == 0) cstart[nb] = (uint32_t)carry;
}

// Moves every entry (and, for the index, its set id) into its bucket.
template <class V, bool INDEX>
__global__ __launch_bounds__(kThreads) void bucket_scatter_kernel(V sets, uint64_t nsets, int shift, int nb,
                                                                  const int64_t* boff, uint32_t* bfill, uint32_t* bu,
                                                                  uint32_t* bs) {
  constexpr int TS = kHistTileSets;
  __shared__ int64_t s_start[TS];
  __shared__ int64_t s_pre[TS + 1];
  __shared__ uint32_t s_wtot[kThreads / 64];
  __shared__ uint32_t h[kBucketMax];  // the tile's entries per bucket, then their next position
  for (uint64_t s0 = (uint64_t)blockIdx.x * TS; s0 < nsets; s0 += (uint64_t)gridDim.x * TS) {
    uint32_t len = 0;
    int64_t start = 0;
    if (threadIdx.x < TS && s0 + threadIdx.x < nsets) {
      start = sets.start(s0 + threadIdx.x);
      len = sets.len(s0 + threadIdx.x);
    }
    for (int i = threadIdx.x; i < nb; i += kThreads) h[i] = 0u;
    tile_prefix<TS>(len, start, s_start, s_pre, s_wtot);
    const int64_t tot = s_pre[TS];
    for (int64_t e = threadIdx.x; e < tot; e += kThreads) {
      const int j = tile_set_of(s_pre, TS, e);
      const uint32_t u = (uint32_t)sets.nodes[s_start[j] + (e - s_pre[j])];
      atomicAdd(&h[u >> shift], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += kThreads)
      if (h[i]) h[i] = (uint32_t)boff[i] + atomicAdd(&bfill[(size_t)i * kLinePad], h[i]);
    __syncthreads();
    for (int64_t e = threadIdx.x; e < tot; e += kThreads) {
      const int j = tile_set_of(s_pre, TS, e);
      const uint32_t u = (uint32_t)sets.nodes[s_start[j] + (e - s_pre[j])];
      const uint32_t pos = atomicAdd(&h[u >> shift], 1u);
      bu[pos] = u;
      if (INDEX) bs[pos] = (uint32_t)(s0 + (uint64_t)j);
    }
    __syncthreads();
  }
}

// The bucket, first entry and end of chunk blockIdx.x; false past the last chunk.
__device__ __forceinline__ bool chunk_of(const int64_t* boff, const uint32_t* cstart, const uint32_t* cb, int nb,
                                         uint32_t& b, int64_t& e0, int64_t& e1, bool& alone) {
  const uint32_t c = blockIdx.x;
  if (c >= cstart[nb]) return false;
  b = cb[c];
  e0 = boff[b] + (int64_t)(c - cstart[b]) * kBucketChunk;
  e1 = min(e0 + (int64_t)kBucketChunk, boff[b + 1]);
  alone = cstart[b + 1] - cstart[b] == 1u;
  return true;
}

// cnt of the chunk's node range: stored where the chunk is its bucket's only
// one, else added with one atomic per node present.
__global__ __launch_bounds__(kThreads) void bucket_count_kernel(const uint32_t* bu, const int64_t* boff,
                                                                const uint32_t* cstart, const uint32_t* cb, int nb,
                                                                int shift, int64_t n, uint32_t* cnt) {
  __shared__ uint32_t lc[1 << kBucketShiftMax];
  uint32_t b;
  int64_t e0, e1;
  bool alone;
  if (!chunk_of(boff, cstart, cb, nb, b, e0, e1, alone)) return;
  const int range = 1 << shift;
  const uint32_t base = b << shift;
  for (int i = threadIdx.x; i < range; i += kThreads) lc[i] = 0u;
  __syncthreads();
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) atomicAdd(&lc[bu[e] - base], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < range && (int64_t)base + i < n; i += kThreads) {
    if (alone) cnt[base + i] = lc[i];
    else if (lc[i]) atomicAdd(&cnt[base + i], lc[i]);
  }
}

// inv_sets of the chunk's nodes: positions from inv_off, plus a base per node
// taken from fill where the bucket has several chunks.
__global__ __launch_bounds__(kThreads) void bucket_index_kernel(const uint32_t* bu, const uint32_t* bs,
                                                                const int64_t* boff, const uint32_t* cstart,
                                                                const uint32_t* cb, int nb, int shift, int64_t n,
                                                                const int64_t* inv_off, uint32_t* fill,
                                                                uint32_t* inv_sets) {
  __shared__ uint32_t lc[1 << kBucketShiftMax];  // the chunk's entries per node, then their next position
  uint32_t b;
  int64_t e0, e1;
  bool alone;
  if (!chunk_of(boff, cstart, cb, nb, b, e0, e1, alone)) return;
  const int range = 1 << shift;
  const uint32_t base = b << shift;
  for (int i = threadIdx.x; i < range; i += kThreads) lc[i] = 0u;
  __syncthreads();
  if (!alone) {
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) atomicAdd(&lc[bu[e] - base], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < range && (int64_t)base + i < n; i += kThreads)
      if (lc[i]) lc[i] = atomicAdd(&fill[base + i], lc[i]);
    __syncthreads();
  }
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
    const uint32_t u = bu[e];
    inv_sets[inv_off[u] + atomicAdd(&lc[u - base], 1u)] = bs[e];
  }
}

// Key of node u: 0 if selected, else count<<32 | (0xFFFFFFFF - u), so the
// maximum key is the largest count with the lowest id; unselected keys > 0.
// Few blocks, 4 nodes per thread and load: one atomicMax per block.
__global__ __launch_bounds__(kThreads) void argmax_kernel(const uint32_t* cnt, const uint8_t* selected, int64_t n,
                                                          unsigned long long* best) {
  unsigned long long key = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n4 = n >> 2;
  const uint4* c4 = reinterpret_cast<const uint4*>(cnt);
  const uint32_t* s4 = reinterpret_cast<const uint32_t*>(selected);
  for (int64_t i = tid; i < n4; i += stride) {
    const uint4 c = c4[i];
    const uint32_t sel = s4[i];
    const uint32_t cv[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const unsigned long long u = (unsigned long long)(4 * i + w);
      const unsigned long long k = ((unsigned long long)cv[w] << 32) | (0xFFFFFFFFull - u);
      if (!((sel >> (8 * w)) & 0xFFu)) key = k > key ? k : key;
    }
  }
  for (int64_t u = 4 * n4 + tid; u < n; u += stride) {
    if (selected[u]) continue;
    const unsigned long long k = ((unsigned long long)cnt[u] << 32) | (0xFFFFFFFFull - (unsigned long long)u);
    key = k > key ? k : key;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(key, o, 64);
    key = y > key ? y : key;
  }
  __shared__ unsigned long long red[kThreads / 64];
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  if (lane == 0) red[wv] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < kThreads / 64; ++w) key = red[w] > key ? red[w] : key;
    if (key) atomicMax(best, key);
  }
}

__device__ __forceinline__ int64_t node_of_key(unsigned long long key) {
  return (int64_t)(0xFFFFFFFFull - (key & 0xFFFFFFFFull));
}

// The chosen node v covers the sets listed in inv_sets[inv_off[v] ..]: mark
// those not covered yet and take them out of the counts of their members
// (v's own count is left alone: v is never chosen again).
template <class V>
__global__ __launch_bounds__(kThreads) void cover_kernel(const unsigned long long* best, const int64_t* inv_off,
                                                         const uint32_t* inv_sets, V sets, uint8_t* covered,
                                                         uint8_t* selected, uint32_t* cnt) {
  __shared__ TileShared<> t;
  if (*best == 0ull) return;  // no unselected node (cannot happen for k <= n)
  const int64_t v = node_of_key(*best);
  if (blockIdx.x == 0 && threadIdx.x == 0) selected[v] = 1u;
  const int64_t lo = inv_off[v], hi = inv_off[v + 1];
  for (int64_t i0 = lo + (int64_t)blockIdx.x * kTileSets; i0 < hi; i0 += (int64_t)gridDim.x * kTileSets) {
    const int ni = (int)min((int64_t)kTileSets, hi - i0);
    // newly covered sets of this tile and their sizes
    uint32_t len = 0;
    int64_t start = 0;
    if (threadIdx.x < ni) {
      const uint32_t sid = inv_sets[i0 + threadIdx.x];
      if (!covered[sid]) {
        covered[sid] = 1u;
        start = sets.start(sid);
        len = sets.len(sid);
      }
    }
    tile_prefix(len, start, t.start, t.pre, t.wtot);
    tile_apply<false>(sets.nodes, t, v, cnt);
  }
}

__global__ void select_kernel(const unsigned long long* best, uint8_t* selected) {
  if (threadIdx.x == 0 && *best != 0ull) selected[node_of_key(*best)] = 1u;
}

// Sets (pool layout) not covered yet that contain the chosen node v: mark
// them and take them out of the counts of their members.
__global__ __launch_bounds__(kThreads) void scan_cover_kernel(const unsigned long long* best, PoolSets sets,
                                                              uint64_t nsets, uint8_t* covered, uint32_t* cnt) {
  __shared__ TileShared<> t;
  __shared__ uint32_t s_hit[kTileSets];
  if (*best == 0ull) return;
  const int64_t v = node_of_key(*best);
  for (uint64_t s0 = (uint64_t)blockIdx.x * kTileSets; s0 < nsets; s0 += (uint64_t)gridDim.x * kTileSets) {
    const int ns = (int)min((uint64_t)kTileSets, nsets - s0);
    uint32_t len = 0;
    int64_t start = 0;
    if (threadIdx.x < ns && !covered[s0 + threadIdx.x]) {
      start = sets.start(s0 + threadIdx.x);
      len = sets.len(s0 + threadIdx.x);
    }
    if (threadIdx.x < kTileSets) s_hit[threadIdx.x] = 0u;
    tile_prefix(len, start, t.start, t.pre, t.wtot);
    // membership of v
    const int64_t tot = t.pre[kTileSets];
    for (int64_t e = threadIdx.x; e < tot; e += kThreads) {
      const int j = tile_set_of(t.pre, kTileSets, e);
      if (sets.nodes[t.start[j] + (e - t.pre[j])] == v) s_hit[j] = 1u;
    }
    __syncthreads();
    bool hit = false;
    if (threadIdx.x < ns) {
      hit = s_hit[threadIdx.x] != 0u;
      if (hit) covered[s0 + threadIdx.x] = 1u;
    }
    tile_prefix(hit ? len : 0u, start, t.start, t.pre, t.wtot);
    tile_apply<false>(sets.nodes, t, v, cnt);
  }
}

unsigned grid_for(uint64_t items, unsigned cap) {
  uint64_t g = (items + kThreads - 1) / kThreads;
  if (g < 1) g = 1;
  return (unsigned)(g > cap ? cap : g);
}

}  // namespace

size_t scan_temp_bytes(uint64_t len) { return ((len + kTile - 1) / kTile + 1) * sizeof(unsigned long long); }

void launch_scan_u32_to_i64(const uint32_t* in, int64_t* out, uint64_t len, void* temp, hipStream_t s) {
  const uint64_t ntiles = (len + kTile - 1) / kTile;
  unsigned long long* ts = static_cast<unsigned long long*>(temp);
  if (ntiles) hipLaunchKernelGGL(scan_tile_sums, dim3((unsigned)ntiles), dim3(kThreads), 0, s, in, len, ts);
  hipLaunchKernelGGL(scan_tile_offsets, dim3(1), dim3(kThreads), 0, s, ts, ntiles, out, len);
  if (ntiles) hipLaunchKernelGGL(scan_apply, dim3((unsigned)ntiles), dim3(kThreads), 0, s, in, len, ts, out);
}

void launch_compact(const int32_t* pool, const uint64_t* set_start, const uint32_t* set_len, const int64_t* out_off,
                    int32_t* out_nodes, uint64_t nsets, hipStream_t s) {
  if (!nsets) return;
  hipLaunchKernelGGL(compact_kernel, dim3(grid_for(nsets, 8192)), dim3(kThreads), 0, s, pool, set_start, set_len,
                     out_off, out_nodes, nsets);
}

void launch_check_ids(const int32_t* nodes, uint64_t total, int64_t n, unsigned int* flag, hipStream_t s) {
  hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, s, flag, (uint64_t)1);
  if (total)
    hipLaunchKernelGGL(check_ids_kernel, dim3(grid_for(total, 4096)), dim3(kThreads), 0, s, nodes, total, n, flag);
}

void launch_set_sizes(const int64_t* set_off, uint32_t* sizes, uint64_t nsets, hipStream_t s) {
  if (!nsets) return;
  hipLaunchKernelGGL(set_sizes_kernel, dim3(grid_for(nsets, 8192)), dim3(kThreads), 0, s, set_off, sizes, nsets);
}

namespace {

CsrSets csr_of(const GreedyArgs& a) { return CsrSets{a.set_off, a.nodes}; }
PoolSets pool_of(const GreedyArgs& a) { return PoolSets{a.set_start, a.set_len, a.nodes}; }

unsigned tile_grid(uint64_t items, uint64_t per_tile) {
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((items + per_tile - 1) / per_tile, 8192));
}

}  // namespace

// ---- the counting sort's workspace ----
namespace {

int bucket_shift(int64_t n) {
  int shift = kBucketShiftMin;
  while (shift <= kBucketShiftMax && ((n + (1ll << shift) - 1) >> shift) > kBucketMax) ++shift;
  return shift;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BucketLayout {
  int shift = 0, nb = 0;
  uint64_t max_chunks = 0;
  size_t bcnt = 0, bcnt_s = 0, bfill = 0, boff = 0, cstart = 0, cb = 0, temp = 0, bu = 0, bs = 0, bytes = 0;
};

// Offsets of the workspace's arrays; bytes == 0 where the collection does not
// fit the counting sort (node ids beyond its ranges, 2^32 entries or more).
BucketLayout bucket_layout(int64_t n, uint64_t total, bool index) {
  BucketLayout L;
  L.shift = bucket_shift(n);
  if (L.shift > kBucketShiftMax || total >= 0xFFFFFFFFull || n < 1) return L;
  L.nb = (int)((n + (1ll << L.shift) - 1) >> L.shift);
  L.max_chunks = (uint64_t)L.nb + total / kBucketChunk + 1;
  size_t at = 0;
  L.bcnt = at;
  at += align256((size_t)L.nb * 4);
  L.bcnt_s = at;
  at += align256((size_t)L.nb * 4 * kLinePad);
  L.bfill = at;
  at += align256((size_t)L.nb * 4 * kLinePad);
  L.boff = at;
  at += align256((size_t)(L.nb + 1) * 8);
  L.cstart = at;
  at += align256((size_t)(L.nb + 1) * 4);
  L.cb = at;
  at += align256((size_t)L.max_chunks * 4);
  L.temp = at;
  at += align256(scan_temp_bytes((uint64_t)L.nb));
  L.bu = at;
  at += align256((size_t)total * 4);
  L.bs = at;
  if (index) at += align256((size_t)total * 4);
  L.bytes = at;
  return L;
}

template <class T>
T* at_offset(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// Sorts the entries into buckets and counts them (cnt zeroed first); with
// `index`, leaves the set ids beside them for bucket_index_kernel.
template <class V>
void bucket_counts(const GreedyArgs& a, V sets, const BucketLayout& L, bool index, hipStream_t s) {
  uint32_t* bcnt = at_offset<uint32_t>(a.bkt, L.bcnt);
  uint32_t* bcnt_s = at_offset<uint32_t>(a.bkt, L.bcnt_s);
  int64_t* boff = at_offset<int64_t>(a.bkt, L.boff);
  uint32_t* cstart = at_offset<uint32_t>(a.bkt, L.cstart);
  uint32_t* cb = at_offset<uint32_t>(a.bkt, L.cb);
  uint32_t* bu = at_offset<uint32_t>(a.bkt, L.bu);
  uint32_t* bs = index ? at_offset<uint32_t>(a.bkt, L.bs) : nullptr;
  // the padded counts and cursors are adjacent: one clear; the scan reads the counts unpadded
  const uint64_t zlen = (uint64_t)(L.bfill - L.bcnt_s) / 4 + (uint64_t)L.nb * kLinePad;
  hipLaunchKernelGGL(zero_u32, dim3(grid_for(zlen, 64)), dim3(kThreads), 0, s, bcnt_s, zlen);
  const unsigned grid = tile_grid(a.nsets, kHistTileSets);
  hipLaunchKernelGGL(bucket_hist_kernel<V>, dim3(grid), dim3(kThreads), 0, s, sets, a.nsets, L.shift, L.nb, bcnt_s);
  hipLaunchKernelGGL(unpad_u32, dim3(grid_for((uint64_t)L.nb, 64)), dim3(kThreads), 0, s, bcnt_s, bcnt, L.nb);
  launch_scan_u32_to_i64(bcnt, boff, (uint64_t)L.nb, at_offset<void>(a.bkt, L.temp), s);
  hipLaunchKernelGGL(bucket_chunks_kernel, dim3(1), dim3(kThreads), 0, s, boff, L.nb, cstart, cb);
  uint32_t* bfill = at_offset<uint32_t>(a.bkt, L.bfill);
  if (index)
    hipLaunchKernelGGL((bucket_scatter_kernel<V, true>), dim3(grid), dim3(kThreads), 0, s, sets, a.nsets, L.shift,
                       L.nb, boff, bfill, bu, bs);
  else
    hipLaunchKernelGGL((bucket_scatter_kernel<V, false>), dim3(grid), dim3(kThreads), 0, s, sets, a.nsets, L.shift,
                       L.nb, boff, bfill, bu, bs);
  hipLaunchKernelGGL(bucket_count_kernel, dim3((unsigned)L.max_chunks), dim3(kThreads), 0, s, bu, boff, cstart, cb,
                     L.nb, L.shift, a.n, a.cnt);
}

}  // namespace

size_t bucket_workspace_bytes(int64_t n, uint64_t total, bool index) { return bucket_layout(n, total, index).bytes; }

void launch_counts(const GreedyArgs& a, hipStream_t s) {
  const uint64_t n = (uint64_t)a.n;
  hipLaunchKernelGGL(zero_u32, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, a.cnt, n);
  if (!a.nsets) return;
  if (a.bkt && a.total) {
    const BucketLayout L = bucket_layout(a.n, a.total, false);
    if (L.bytes) {
      if (a.set_off) bucket_counts(a, csr_of(a), L, false, s);
      else bucket_counts(a, pool_of(a), L, false, s);
      return;
    }
  }
  if (a.set_off) {
    if (a.total)
      hipLaunchKernelGGL(hist_flat_kernel, dim3(tile_grid(a.total, kTileEntries)), dim3(kThreads), 0, s, a.nodes,
                         a.total, a.cnt);
  } else {
    hipLaunchKernelGGL(hist_sets_kernel<PoolSets>, dim3(tile_grid(a.nsets, kHistTileSets)), dim3(kThreads), 0, s,
                       pool_of(a), a.nsets, a.cnt);
  }
}

void launch_index(const GreedyArgs& a, hipStream_t s) {
  const uint64_t n = (uint64_t)a.n;
  if (a.bkt && a.nsets && a.total) {
    const BucketLayout L = bucket_layout(a.n, a.total, true);
    if (L.bytes) {
      hipLaunchKernelGGL(zero_u32, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, a.cnt, n);
      if (a.set_off) bucket_counts(a, csr_of(a), L, true, s);
      else bucket_counts(a, pool_of(a), L, true, s);
      hipLaunchKernelGGL(zero_u32, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, a.fill, n);
      launch_scan_u32_to_i64(a.cnt, a.inv_off, n, a.scan_temp, s);
      hipLaunchKernelGGL(bucket_index_kernel, dim3((unsigned)L.max_chunks), dim3(kThreads), 0, s,
                         at_offset<uint32_t>(a.bkt, L.bu), at_offset<uint32_t>(a.bkt, L.bs),
                         at_offset<int64_t>(a.bkt, L.boff), at_offset<uint32_t>(a.bkt, L.cstart),
                         at_offset<uint32_t>(a.bkt, L.cb), L.nb, L.shift, a.n, a.inv_off, a.fill, a.inv_sets);
      return;
    }
  }
  launch_counts(a, s);
  hipLaunchKernelGGL(zero_u32, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, a.fill, n);
  launch_scan_u32_to_i64(a.cnt, a.inv_off, n, a.scan_temp, s);
  if (!a.nsets) return;
  const unsigned grid = tile_grid(a.nsets, kTileSets);
  if (a.set_off)
    hipLaunchKernelGGL(scatter_kernel<CsrSets>, dim3(grid), dim3(kThreads), 0, s, csr_of(a), a.nsets, a.inv_off,
                       a.fill, a.inv_sets);
  else
    hipLaunchKernelGGL(scatter_kernel<PoolSets>, dim3(grid), dim3(kThreads), 0, s, pool_of(a), a.nsets, a.inv_off,
                       a.fill, a.inv_sets);
}

void launch_zero_counts(uint32_t* cnt, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero_u32, dim3(grid_for((uint64_t)n, 4096)), dim3(kThreads), 0, s, cnt, (uint64_t)n);
}

void launch_greedy_init(const GreedyArgs& a, uint64_t covered_len, int k, hipStream_t s) {
  const uint64_t n = (uint64_t)a.n;
  if (covered_len)
    hipLaunchKernelGGL(zero_u8, dim3(grid_for(covered_len, 4096)), dim3(kThreads), 0, s, a.covered, covered_len);
  hipLaunchKernelGGL(zero_u8, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, a.selected, n);
  hipLaunchKernelGGL(zero_u64, dim3(1), dim3(kThreads), 0, s, a.best, (uint64_t)k);
}

namespace {
void launch_argmax(const GreedyArgs& a, int j, hipStream_t s) {
  const uint64_t n4 = ((uint64_t)a.n + 3) / 4;
  hipLaunchKernelGGL(argmax_kernel, dim3(grid_for(n4, 256)), dim3(kThreads), 0, s, a.cnt, a.selected, a.n,
                     a.best + j);
}
}  // namespace

void launch_argmax_step(const GreedyArgs& a, int j, hipStream_t s) {
  launch_argmax(a, j, s);
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(64), 0, s, a.best + j, a.selected);
}

void launch_cover_step(const GreedyArgs& a, int j, hipStream_t s) {
  if (!a.nsets) {
    // nothing to cover, but the choice must still leave the candidates
    hipLaunchKernelGGL(select_kernel, dim3(1), dim3(64), 0, s, a.best + j, a.selected);
    return;
  }
  // the chosen node's list holds at most nsets sets: no more blocks than its tiles
  const dim3 grid((unsigned)std::min<uint64_t>(1024, (a.nsets + kTileSets - 1) / kTileSets));
  if (a.set_off)
    hipLaunchKernelGGL(cover_kernel<CsrSets>, grid, dim3(kThreads), 0, s, a.best + j, a.inv_off, a.inv_sets,
                       csr_of(a), a.covered, a.selected, a.cnt);
  else
    hipLaunchKernelGGL(cover_kernel<PoolSets>, grid, dim3(kThreads), 0, s, a.best + j, a.inv_off, a.inv_sets,
                       pool_of(a), a.covered, a.selected, a.cnt);
}

void launch_pool_hist(const int32_t* pool, const uint64_t* set_start, const uint32_t* set_len, uint64_t nsets,
                      uint32_t* cnt, hipStream_t s) {
  if (!nsets) return;
  hipLaunchKernelGGL(hist_sets_kernel<PoolSets>, dim3(tile_grid(nsets, kHistTileSets)), dim3(kThreads), 0, s,
                     PoolSets{set_start, set_len, pool}, nsets, cnt);
}

void launch_pool_cover(const unsigned long long* best, const int32_t* pool, const uint64_t* set_start,
                       const uint32_t* set_len, uint64_t nsets, uint8_t* covered, uint32_t* cnt, hipStream_t s) {
  if (!nsets) return;
  hipLaunchKernelGGL(scan_cover_kernel, dim3(tile_grid(nsets, kTileSets)), dim3(kThreads), 0, s, best,
                     PoolSets{set_start, set_len, pool}, nsets, covered, cnt);
}

// ---- a greedy that allocates nothing ----
//
// For callers that cannot allocate device memory (under HIP graph capture, in
// serving loops), the greedy's work arrays can live in one fixed device array
// instead of context buffers.  Each GPU holds its own copy at its own
// address, found once per device with hipGetSymbolAddress; in host code the
// array's name is not a device address, so only that address is ever used.
namespace {
constexpr size_t kStaticCnt = 0;                                             // uint32 [kStaticMaxN]
constexpr size_t kStaticFill = kStaticCnt + 4 * kStaticMaxN;                 // uint32 [kStaticMaxN]
constexpr size_t kStaticInvOff = kStaticFill + 4 * kStaticMaxN;              // int64 [kStaticMaxN + 1]
constexpr size_t kStaticInvSets = kStaticInvOff + 8 * (kStaticMaxN + 64);   // uint32 [kStaticMaxEntries]
constexpr size_t kStaticCovered = kStaticInvSets + 4 * kStaticMaxEntries;    // uint8 [kStaticMaxSets]
constexpr size_t kStaticSelected = kStaticCovered + kStaticMaxSets;          // uint8 [kStaticMaxN]
constexpr size_t kStaticBest = kStaticSelected + kStaticMaxN;                // uint64 [kStaticMaxK]
constexpr size_t kStaticMisc = kStaticBest + 8 * kStaticMaxK;                // id-check flag, an empty CSR offset
constexpr size_t kStaticScan = kStaticMisc + 256;                            // scan tile sums
constexpr size_t kStaticBytes = kStaticScan + ((kStaticMaxN + 1 + kTile - 1) / kTile + 1) * 8 + 256;
static_assert(kStaticInvSets % 256 == 0 && kStaticBest % 8 == 0, "alignment");

__device__ __align__(256) unsigned char scratch[kStaticBytes];

std::mutex g_static_mu;
void* g_static_ptr[kStaticMaxDevices] = {};

__global__ void set_u64_kernel(unsigned long long* p, unsigned long long v) {
  if (threadIdx.x == 0) *p = v;
}
}  // namespace

size_t static_scratch_bytes() { return kStaticBytes; }

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kStaticMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (g_static_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_static_ptr[device] = ptr;
  return hipSuccess;
}

StaticGreedy static_greedy_layout(int device) {
  StaticGreedy st;
  memset(&st, 0, sizeof(st));
  void* base = nullptr;
  if (device >= 0 && device < kStaticMaxDevices) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    base = g_static_ptr[device];
  }
  if (!base) return st;
  unsigned char* b = static_cast<unsigned char*>(base);
  st.cnt = reinterpret_cast<uint32_t*>(b + kStaticCnt);
  st.fill = reinterpret_cast<uint32_t*>(b + kStaticFill);
  st.inv_off = reinterpret_cast<int64_t*>(b + kStaticInvOff);
  st.inv_sets = reinterpret_cast<uint32_t*>(b + kStaticInvSets);
  st.covered = b + kStaticCovered;
  st.selected = b + kStaticSelected;
  st.best = reinterpret_cast<unsigned long long*>(b + kStaticBest);
  st.flag = reinterpret_cast<unsigned int*>(b + kStaticMisc);
  st.zero_off = reinterpret_cast<int64_t*>(b + kStaticMisc + 8);
  st.scan_temp = b + kStaticScan;
  return st;
}

void launch_set_u64(unsigned long long* p, unsigned long long v, hipStream_t s) {
  hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, s, p, v);
}

void launch_greedy(const GreedyArgs& a, int k, hipStream_t s) {
  launch_greedy_init(a, a.nsets, k, s);
  for (int j = 0; j < k; ++j) {
    launch_argmax(a, j, s);
    // the last choice changes no later step: its cover pass is skipped
    if (j + 1 < k) launch_cover_step(a, j, s);
  }
}

}  // namespace tim
