// RR collection layout and greedy maximum coverage on gfx950.
//
// Compaction (scan of set sizes, then a gather) turns the node pool written by
// the samplers into a flat CSR of sets in set-id order.  A counting sort of
// that CSR (histogram, scan, scatter) builds the node -> sets inverted index;
// its histogram is also the initial coverage count of every node.  The greedy
// of Algorithm 1 (lines 3-7) then runs on the device without host round
// trips: per step one argmax kernel packs (count, ~id) into a 64-bit key so
// that a single atomicMax selects the largest count with ties to the lowest
// id, and one cover kernel marks the chosen node's uncovered sets and
// decrements the counts of their members.
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

// cnt[u] = number of sets containing u (sets never repeat a node).
__global__ void hist_kernel(const int64_t* set_off, const int32_t* nodes, uint64_t nsets, uint32_t* cnt) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nsets; s += stride)
    for (int64_t i = set_off[s]; i < set_off[s + 1]; ++i) atomicAdd(&cnt[nodes[i]], 1u);
}

__global__ void scatter_kernel(const int64_t* set_off, const int32_t* nodes, uint64_t nsets, const int64_t* inv_off,
                               uint32_t* fill, uint32_t* inv_sets) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nsets; s += stride)
    for (int64_t i = set_off[s]; i < set_off[s + 1]; ++i) {
      const int32_t u = nodes[i];
      inv_sets[inv_off[u] + atomicAdd(&fill[u], 1u)] = (uint32_t)s;
    }
}

// Key of node u: 0 if selected, else count<<32 | (0xFFFFFFFF - u), so the
// maximum key is the largest count with the lowest id; unselected keys > 0.
__global__ __launch_bounds__(kThreads) void argmax_kernel(const uint32_t* cnt, const uint8_t* selected, int64_t n,
                                                          unsigned long long* best) {
  unsigned long long key = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
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
    for (int w = 1; w < kThreads / 64; ++w) key = red[w] > key ? red[w] : key;
    key = red[0] > key ? red[0] : key;
    if (key) atomicMax(best, key);
  }
}

__global__ void cover_kernel(const unsigned long long* best, const int64_t* inv_off, const uint32_t* inv_sets,
                             const int64_t* set_off, const int32_t* nodes, uint8_t* covered, uint8_t* selected,
                             uint32_t* cnt) {
  if (*best == 0ull) return;  // no unselected node (cannot happen for k <= n)
  const int64_t v = (int64_t)(0xFFFFFFFFull - (*best & 0xFFFFFFFFull));
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) selected[v] = 1u;
  const int64_t lo = inv_off[v], hi = inv_off[v + 1];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = lo + (int64_t)gid; i < hi; i += stride) {
    const uint32_t s = inv_sets[i];
    if (covered[s]) continue;
    covered[s] = 1u;
    for (int64_t t = set_off[s]; t < set_off[s + 1]; ++t) atomicSub(&cnt[nodes[t]], 1u);
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

void launch_index(const GreedyArgs& a, hipStream_t s) {
  const uint64_t n = (uint64_t)a.n;
  hipLaunchKernelGGL(zero_u32, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, a.cnt, n);
  hipLaunchKernelGGL(zero_u32, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, a.fill, n);
  if (a.nsets)
    hipLaunchKernelGGL(hist_kernel, dim3(grid_for(a.nsets, 8192)), dim3(kThreads), 0, s, a.set_off, a.nodes, a.nsets,
                       a.cnt);
  launch_scan_u32_to_i64(a.cnt, a.inv_off, n, a.scan_temp, s);
  if (a.nsets)
    hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(a.nsets, 8192)), dim3(kThreads), 0, s, a.set_off, a.nodes,
                       a.nsets, a.inv_off, a.fill, a.inv_sets);
}

void launch_greedy(const GreedyArgs& a, int k, hipStream_t s) {
  const uint64_t n = (uint64_t)a.n;
  if (a.nsets) hipLaunchKernelGGL(zero_u8, dim3(grid_for(a.nsets, 4096)), dim3(kThreads), 0, s, a.covered, a.nsets);
  hipLaunchKernelGGL(zero_u8, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, a.selected, n);
  hipLaunchKernelGGL(zero_u64, dim3(1), dim3(kThreads), 0, s, a.best, (uint64_t)k);
  const unsigned gmax = grid_for(n, 2048);
  for (int j = 0; j < k; ++j) {
    hipLaunchKernelGGL(argmax_kernel, dim3(gmax), dim3(kThreads), 0, s, a.cnt, a.selected, a.n, a.best + j);
    hipLaunchKernelGGL(cover_kernel, dim3(1024), dim3(kThreads), 0, s, a.best + j, a.inv_off, a.inv_sets, a.set_off,
                       a.nodes, a.covered, a.selected, a.cnt);
  }
}

}  // namespace tim
