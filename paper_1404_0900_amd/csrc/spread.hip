// Spread evaluation by forward Monte-Carlo runs: E[I(S)] in the live-edge view
// of Section 2.2, estimated as the paper's experiments do it (Section 7) by
// the mean spread over independent runs.  Run r is the live-edge world of
// phase 65 and set id r: IC edge e is live iff its coin word (kind 1, group
// e >> 2, word e & 3) is at most its threshold, and in LT node v's live
// in-edge is the one its pick draw (kind 2, index v) selects, and under the
// general triggering model v's live in-edges are the set its draw of kind 3
// selects - the same rules the RR-set samplers use (pick.hpp).  A run's spread is the number of nodes
// reachable from S along live edges, found by a forward BFS over the graph's
// out-edge lists (built once from the in-CSR and kept with the graph).
#include "engine.hpp"
#include "pick.hpp"
#include "rng.hpp"

namespace tim {
namespace {

constexpr int kThreads = 256;
constexpr int kWave = 64;
constexpr uint32_t kPhaseEval = 65;

__global__ void out_count_kernel(const int32_t* src, int64_t m, uint32_t* cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) atomicAdd(&cnt[src[e]], 1u);
}

// In-edge e (into v, the largest node with in_off[v] <= e) joins the out-list
// of its source as (v, e); the order inside an out-list is not defined.
__global__ void out_scatter_kernel(const int64_t* in_off, const int32_t* src, int64_t n, int64_t m,
                                   const int64_t* out_off, uint32_t* fill, int32_t* out_dst, uint32_t* out_eid) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (in_off[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    const int32_t u = src[e];
    const int64_t pos = out_off[u] + (int64_t)atomicAdd(&fill[u], 1u);
    out_dst[pos] = (int32_t)lo;
    out_eid[pos] = (uint32_t)e;
  }
}

__device__ __forceinline__ unsigned long long wave_incl_scan64(unsigned long long x, int lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

// One block per slot; the block takes runs from a counter until they run out.
template <int MODEL, bool WC>
__global__ __launch_bounds__(kThreads) void spread_kernel(SpreadArgs a) {
  __shared__ unsigned long long s_incl[kThreads];
  __shared__ int64_t s_ea[kThreads];
  __shared__ unsigned long long s_wtot[kThreads / kWave];
  __shared__ unsigned long long s_idx;
  __shared__ uint32_t s_tail, s_epoch;
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  const GraphView g = a.g;
  const Key key = make_key(a.seed);
  const int slot = blockIdx.x;
  uint32_t* stamp = a.stamp + (size_t)slot * (size_t)a.stride;
  int32_t* queue = a.queue + (size_t)slot * (size_t)a.stride;
  unsigned long long total = 0;
  for (;;) {
    if (tid == 0) {
      s_idx = atomicAdd(&a.ctr[0], 1ull);
      s_epoch = a.epoch[slot] + 1u;
      s_tail = 0u;
    }
    __syncthreads();
    const unsigned long long idx = s_idx;
    if (idx >= a.runs) break;
    uint32_t ep = s_epoch;
    if (ep == 0u) {  // stamp counter wrapped: start the slot afresh
      for (uint64_t i = tid; i < a.stride; i += kThreads) stamp[i] = 0u;
      ep = 1u;
    }
    __syncthreads();
    if (tid == 0) a.epoch[slot] = ep;
    const SetStream st = make_set_stream(kPhaseEval, a.first + idx);
    for (int i = tid; i < a.nseeds; i += kThreads) {
      const int32_t u = a.seeds[i];
      if (atomicExch(&stamp[u], ep) != ep) queue[atomicAdd(&s_tail, 1u)] = u;
    }
    __syncthreads();
    uint32_t head = 0;
    for (;;) {
      const uint32_t tail = s_tail;
      if (head >= tail) break;
      const int nb = (int)min(tail - head, (uint32_t)kThreads);
      int64_t ea = 0;
      unsigned long long d = 0;
      if (tid < nb) {
        const int32_t u = queue[head + tid];
        ea = a.out_off[u];
        d = (unsigned long long)(a.out_off[u + 1] - ea);
      }
      unsigned long long incl = wave_incl_scan64(d, lane);
      if (lane == kWave - 1) s_wtot[wv] = incl;
      __syncthreads();
      for (int w = 0; w < wv; ++w) incl += s_wtot[w];
      s_incl[tid] = incl;
      s_ea[tid] = ea;
      __syncthreads();
      const unsigned long long items = s_incl[kThreads - 1];
      head += (uint32_t)nb;
      for (unsigned long long item = tid; item < items; item += kThreads) {
        int lo = 0, hi = nb - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (s_incl[mid] > item) hi = mid;
          else lo = mid + 1;
        }
        const unsigned long long excl = lo ? s_incl[lo - 1] : 0ull;
        const int64_t x = s_ea[lo] + (int64_t)(item - excl);
        const int32_t v = a.out_dst[x];
        if (stamp[v] == ep) continue;
        const int64_t e = (int64_t)a.out_eid[x];
        const int64_t iv = g.off[v];
        const int64_t din = g.off[v + 1] - iv;
        bool live;
        if (MODEL == 0) {
          const uint4 c = draw(key, st, kKindCoin, (uint64_t)e >> 2);
          const uint32_t words[4] = {c.x, c.y, c.z, c.w};
          live = edge_live<WC>(words[e & 3], WC ? 0u : g.thr[e], din);
        } else if (MODEL == 2) {
          // general triggering: e is live iff it belongs to the set v draws
          const int64_t j = trig_pick(g, key, st, v);
          live = false;
          if (j >= 0)
            for (int64_t i = g.tset[j]; i < g.tset[j + 1]; ++i) live = live || iv + (int64_t)g.tmem[i] == e;
        } else {
          live = lt_pick_edge(g, key, st, v, iv, din) == e;
        }
        if (live && atomicExch(&stamp[v], ep) != ep) queue[atomicAdd(&s_tail, 1u)] = v;
      }
      __syncthreads();
    }
    if (tid == 0) {
      const uint32_t cnt = s_tail;
      if (a.counts) a.counts[idx] = cnt;
      total += cnt;
    }
    __syncthreads();
  }
  if (tid == 0 && total) atomicAdd(&a.ctr[1], total);
}

}  // namespace

void launch_out_csr_count(const int32_t* src, int64_t m, uint32_t* cnt, hipStream_t s) {
  hipLaunchKernelGGL(out_count_kernel, dim3(2048), dim3(kThreads), 0, s, src, m, cnt);
}

void launch_out_csr_scatter(const int64_t* in_off, const int32_t* src, int64_t n, int64_t m, const int64_t* out_off,
                            uint32_t* fill, int32_t* out_dst, uint32_t* out_eid, hipStream_t s) {
  hipLaunchKernelGGL(out_scatter_kernel, dim3(2048), dim3(kThreads), 0, s, in_off, src, n, m, out_off, fill, out_dst,
                     out_eid);
}

void launch_spread(int model, const SpreadArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)a.slots), blk(kThreads);
  if (model == 0) {
    if (a.g.thr) hipLaunchKernelGGL((spread_kernel<0, false>), grid, blk, 0, s, a);
    else hipLaunchKernelGGL((spread_kernel<0, true>), grid, blk, 0, s, a);
  } else if (model == 2) {
    hipLaunchKernelGGL((spread_kernel<2, false>), grid, blk, 0, s, a);
  } else {
    hipLaunchKernelGGL((spread_kernel<1, false>), grid, blk, 0, s, a);
  }
}

}  // namespace tim
