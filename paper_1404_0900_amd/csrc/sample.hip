// RR-set samplers for gfx950 (Definitions 1-2; Section 3.1; Section 4.2).
//
// IC, wave-level pass: one 64-wide wavefront builds one RR set at a time by
// reverse BFS.  The set's nodes live in an LDS queue (which is also the
// output list) and an LDS open-addressing hash marks visited nodes.  Each BFS
// step takes up to 64 queued nodes, prefix-sums the number of 4-edge groups
// of their in-edge lists, and spreads the groups over the lanes: a lane loads
// 4 consecutive sources with one 16-byte load, draws one Philox block for the
// group and decides the 4 edges with its 4 words.  Live edges into unvisited
// nodes are appended to the queue.  Sets that outgrow the LDS structures are
// handed to the large-set pass (deterministic: a set is a pure function of its
// keys, so restarting it elsewhere gives the same set).
//
// LT, lane-level pass: each lane walks one set's chain (one live in-edge per
// node); the chain sits in LDS with a 64-bit membership signature in a
// register; longer chains go to the large-set pass.
//
// Large-set pass: a 256-thread block per IC set (lane per set for LT) with a
// visited-stamp array and a queue of n entries per slot in device memory.
//
// Each launch also reduces what the phase needs: the exact 128-bit sum of
// kappa(R) * 2^53 (Equation (8)), the widths (Equation (1)), the set sizes,
// and the number of sets meeting a seed set (Algorithm 3, line 10).
#include "engine.hpp"
#include "rng.hpp"

namespace tim {
namespace {

constexpr int kWave = 64;
constexpr int kIcWaves = 4;        // wavefronts per block, IC wave-level pass
constexpr int kQCap = 512;         // nodes of one set held in LDS
constexpr int kHLog = 10;
constexpr int kHCap = 1 << kHLog;  // LDS hash slots per wavefront
constexpr int kLtWaves = 2;        // wavefronts per block, LT lane-level pass
constexpr int kChain = 64;         // LT chain length held in LDS
constexpr int kBigThreads = 256;   // IC large-set pass block size

typedef unsigned __int128 u128;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// kappa(R) * 2^53 (Equation (8)): q = 1 - w/m, q^k by binary exponentiation,
// every operation a correctly rounded binary64 operation.  kappa is a
// multiple of 2^-53 in [0, 1], so the scaled value is an exact integer.
__device__ __forceinline__ uint64_t kappa_fixed(uint64_t w, int64_t m, int k) {
  const double q = __dsub_rn(1.0, __ddiv_rn((double)w, (double)m));
  double r = 1.0, b = q;
  unsigned int e = (unsigned int)k;
  while (e) {
    if (e & 1u) r = __dmul_rn(r, b);
    e >>= 1;
    if (e) b = __dmul_rn(b, b);
  }
  return (uint64_t)__dmul_rn(__dsub_rn(1.0, r), 9007199254740992.0);
}

__device__ __forceinline__ void add_u128(unsigned long long* lohi, u128 v) {
  const unsigned long long lo = (unsigned long long)v;
  unsigned long long hi = (unsigned long long)(v >> 64);
  if (lo) {
    const unsigned long long old = atomicAdd(&lohi[0], lo);
    if (old + lo < old) hi += 1ull;
  }
  if (hi) atomicAdd(&lohi[1], hi);
}

__device__ __forceinline__ bool in_seed(const uint32_t* bits, int32_t u) {
  return (bits[(uint32_t)u >> 5] >> ((uint32_t)u & 31u)) & 1u;
}

// Edge e of an in-list of length d decided by word x: live iff x <= t(e).
template <bool WC>
__device__ __forceinline__ bool edge_live(uint32_t x, uint32_t t, int64_t d) {
  if (WC) {
    // t = floor(2^32/d) - 1, and x <= t  <=>  (x + 1) * d <= 2^32
    return (uint64_t)((uint64_t)x + 1ull) * (uint64_t)d <= (1ull << 32);
  } else {
    return x <= t;
  }
}

// Open addressing in LDS, key u+1 (0 = empty).  1: inserted, 0: present, -1: full.
__device__ __forceinline__ int lds_insert(uint32_t* h, uint32_t u) {
  const uint32_t key = u + 1u;
  uint32_t pos = (u * 0x9E3779B1u) >> (32 - kHLog);
  for (int i = 0; i < kHCap; ++i) {
    const uint32_t cur = h[pos];
    if (cur == key) return 0;
    if (cur == 0u) {
      const uint32_t old = atomicCAS(&h[pos], 0u, key);
      if (old == 0u) return 1;
      if (old == key) return 0;
    }
    pos = (pos + 1u) & (kHCap - 1u);
  }
  return -1;
}

struct Acc {
  u128 kappa = 0;
  unsigned long long width = 0, nodes = 0, covered = 0;
};

__device__ __forceinline__ void flush(const SampleArgs& a, const Acc& acc) {
  add_u128(&a.ctr[kCtrKappaLo], acc.kappa);
  if (acc.width) atomicAdd(&a.ctr[kCtrWidth], acc.width);
  if (acc.nodes) atomicAdd(&a.ctr[kCtrNodes], acc.nodes);
  if (acc.covered) atomicAdd(&a.ctr[kCtrCovered], acc.covered);
}

__device__ __forceinline__ void defer(const SampleArgs& a, uint64_t rel) {
  const unsigned long long pos = atomicAdd(&a.ctr[kCtrDeferred], 1ull);
  if (pos < a.deferred_cap) a.deferred[pos] = rel;
}

// ------------------------------------------------------------------------
// IC, wave-level pass.
// ------------------------------------------------------------------------
template <int MODE, bool WC>
__global__ __launch_bounds__(kIcWaves* kWave) void ic_wave_kernel(SampleArgs a) {
  __shared__ int32_t s_queue[kIcWaves][kQCap];
  __shared__ uint32_t s_hash[kIcWaves][kHCap];
  __shared__ uint32_t s_tail[kIcWaves];
  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  int32_t* q = s_queue[wv];
  uint32_t* h = s_hash[wv];
  const GraphView g = a.g;
  Acc acc;

  unsigned long long rel = 0;
  if (lane == 0) rel = atomicAdd(&a.ctr[kCtrNextSet], 1ull);
  rel = __shfl(rel, 0);
  while (rel < a.count) {
    unsigned long long next = 0;
    if (lane == 0) next = atomicAdd(&a.ctr[kCtrNextSet], 1ull);
    const SetStream st = make_set_stream(a.seed, a.phase, a.first + rel);

    uint4* h4 = reinterpret_cast<uint4*>(h);
    for (int i = lane; i < kHCap / 4; i += kWave) h4[i] = make_uint4(0u, 0u, 0u, 0u);
    const int32_t root = draw_root(st, g.n);
    wave_sync();
    if (lane == 0) {
      q[0] = root;
      s_tail[wv] = 1u;
      lds_insert(h, (uint32_t)root);
    }
    wave_sync();

    bool hit = (MODE == kModeCover) && in_seed(a.seed_bits, root);
    bool bad = false;
    int head = 0, tail = 1;
    unsigned long long wlane = 0;
    while (head < tail && !hit && !bad) {
      const int nb = min(tail - head, kWave);
      int64_t ea = 0;
      int64_t d = 0;
      uint32_t ng = 0;
      if (lane < nb) {
        const int32_t v = q[head + lane];
        ea = g.off[v];
        const int64_t eb = g.off[v + 1];
        d = eb - ea;
        ng = d ? (uint32_t)(((eb - 1) >> 2) - (ea >> 2) + 1) : 0u;
      }
      wlane += (unsigned long long)d;
      head += nb;
      const uint32_t incl = wave_incl_scan(ng, lane);
      const uint32_t excl = incl - ng;
      const uint32_t total = __shfl(incl, kWave - 1);
      bool lhit = false, lbad = false;
      for (uint32_t base = 0; base < total; base += kWave) {
        const uint32_t item = base + (uint32_t)lane;
        // owner = number of lanes whose inclusive count is <= item
        int owner = 0;
#pragma unroll
        for (int step = kWave / 2; step > 0; step >>= 1) {
          const uint32_t c = __shfl(incl, owner + step - 1);
          if (c <= item) owner += step;
        }
        owner = min(owner, kWave - 1);
        const int64_t oa = __shfl(ea, owner);
        const int64_t od = __shfl(d, owner);
        const uint32_t oex = __shfl(excl, owner);
        if (item < total) {
          const int64_t grp = (oa >> 2) + (int64_t)(item - oex);
          const int4 s4 = reinterpret_cast<const int4*>(g.src)[grp];
          uint4 t4 = make_uint4(0u, 0u, 0u, 0u);
          if (!WC) t4 = reinterpret_cast<const uint4*>(g.thr)[grp];
          const uint4 x = draw(st, kKindCoin, (uint64_t)grp);
          const int32_t sv[4] = {s4.x, s4.y, s4.z, s4.w};
          const uint32_t xv[4] = {x.x, x.y, x.z, x.w};
          const uint32_t tv[4] = {t4.x, t4.y, t4.z, t4.w};
          const int64_t e0 = grp << 2;
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int64_t e = e0 + w;
            if (e < oa || e >= oa + od) continue;
            if (!edge_live<WC>(xv[w], tv[w], od)) continue;
            const int32_t u = sv[w];
            const int r = lds_insert(h, (uint32_t)u);
            if (r < 0) {
              lbad = true;
            } else if (r == 1) {
              const uint32_t pos = atomicAdd(&s_tail[wv], 1u);
              if (pos < (uint32_t)kQCap) q[pos] = u;
              else lbad = true;
              if (MODE == kModeCover && in_seed(a.seed_bits, u)) lhit = true;
            }
          }
        }
      }
      wave_sync();
      tail = (int)min(s_tail[wv], (uint32_t)kQCap + 1u);
      hit = __any(lhit);
      bad = __any(lbad);
    }

    if (bad) {
      if (lane == 0) defer(a, rel);
    } else {
      const unsigned long long width = wave_sum(wlane);
      if (MODE == kModeWidth) {
        if (lane == 0) {
          acc.kappa += kappa_fixed(width, g.m, a.k);
          acc.width += width;
          acc.nodes += (unsigned long long)tail;
          if (a.widths) a.widths[rel] = width;
          if (a.sizes) a.sizes[rel] = (uint32_t)tail;
        }
      } else if (MODE == kModeEmit) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&a.ctr[kCtrPoolCursor], (unsigned long long)tail);
        base = __shfl(base, 0);
        if (base + (unsigned long long)tail <= a.pool_cap)
          for (int i = lane; i < tail; i += kWave) a.pool[base + i] = q[i];
        if (lane == 0) {
          a.set_start[rel] = base;
          a.set_len[rel] = (uint32_t)tail;
          if (a.widths) a.widths[rel] = width;
          acc.width += width;
          acc.nodes += (unsigned long long)tail;
        }
      } else {
        if (lane == 0 && hit) acc.covered += 1;
      }
    }
    rel = __shfl(next, 0);
    wave_sync();
  }
  if (lane == 0) flush(a, acc);
}

// ------------------------------------------------------------------------
// LT, lane-level pass: one chain per lane.
// ------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sig_bit(int32_t u) { return 1ull << (((uint32_t)u * 0x9E3779B1u) >> 26); }

template <int MODE>
__global__ __launch_bounds__(kLtWaves* kWave) void lt_lane_kernel(SampleArgs a) {
  __shared__ int32_t s_chain[kLtWaves][kChain][kWave];
  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  int32_t(*chain)[kWave] = s_chain[wv];
  const GraphView g = a.g;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  Acc acc;

  bool active = false, exhausted = false, hit = false;
  unsigned long long rel = 0, width = 0;
  int32_t v = 0;
  int len = 0;
  uint64_t sig = 0;
  SetStream st = make_set_stream(a.seed, a.phase, a.first);
  for (;;) {
    const bool want = !active && !exhausted;
    const uint64_t wmask = __ballot(want);
    if (wmask) {
      const int leader = __ffsll((unsigned long long)wmask) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(&a.ctr[kCtrNextSet], (unsigned long long)__popcll(wmask));
      base = __shfl(base, leader);
      if (want) {
        rel = base + (unsigned long long)__popcll(wmask & below);
        if (rel >= a.count) {
          exhausted = true;
        } else {
          st = make_set_stream(a.seed, a.phase, a.first + rel);
          v = draw_root(st, g.n);
          chain[0][lane] = v;
          len = 1;
          width = 0;
          sig = sig_bit(v);
          hit = (MODE == kModeCover) && in_seed(a.seed_bits, v);
          active = true;
        }
      }
    }
    if (__ballot(active) == 0) break;
    if (!active) continue;
    bool done = hit, bad = false;
    if (!done) {
      const int64_t ea = g.off[v];
      const int64_t d = g.off[v + 1] - ea;
      width += (unsigned long long)d;
      if (d == 0) {
        done = true;
      } else {
        const uint64_t j = scale64(draw(st, kKindPick, (uint64_t)v), (uint64_t)d);
        const int32_t u = g.src[ea + (int64_t)j];
        const uint64_t bit = sig_bit(u);
        bool seen = false;
        if (sig & bit) {
          for (int i = 0; i < len; ++i) {
            if (chain[i][lane] == u) { seen = true; break; }
          }
        }
        if (seen) {
          done = true;
        } else if (len == kChain) {
          bad = true;
          done = true;
        } else {
          chain[len][lane] = u;
          ++len;
          sig |= bit;
          v = u;
          if (MODE == kModeCover && in_seed(a.seed_bits, u)) {
            hit = true;
            done = true;
          }
        }
      }
    }
    if (done) {
      active = false;
      if (bad) {
        defer(a, rel);
      } else if (MODE == kModeWidth) {
        acc.kappa += kappa_fixed(width, g.m, a.k);
        acc.width += width;
        acc.nodes += (unsigned long long)len;
        if (a.widths) a.widths[rel] = width;
        if (a.sizes) a.sizes[rel] = (uint32_t)len;
      } else if (MODE == kModeEmit) {
        const unsigned long long base = atomicAdd(&a.ctr[kCtrPoolCursor], (unsigned long long)len);
        if (base + (unsigned long long)len <= a.pool_cap)
          for (int i = 0; i < len; ++i) a.pool[base + i] = chain[i][lane];
        a.set_start[rel] = base;
        a.set_len[rel] = (uint32_t)len;
        if (a.widths) a.widths[rel] = width;
        acc.width += width;
        acc.nodes += (unsigned long long)len;
      } else if (hit) {
        acc.covered += 1;
      }
    }
  }
  flush(a, acc);
}

// ------------------------------------------------------------------------
// Large-set pass.
// ------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long deferred_count(const SampleArgs& a) {
  const unsigned long long d = a.ctr[kCtrDeferred];
  return d < a.deferred_cap ? d : a.deferred_cap;
}

// IC: one 256-thread block per set, visited stamps and queue in device memory.
template <int MODE, bool WC>
__global__ __launch_bounds__(kBigThreads) void ic_big_kernel(SampleArgs a) {
  constexpr int T = kBigThreads;
  __shared__ uint32_t s_incl[T];
  __shared__ int64_t s_ea[T];
  __shared__ int64_t s_d[T];
  __shared__ uint32_t s_wtot[T / kWave];
  __shared__ unsigned long long s_red[T / kWave];
  __shared__ unsigned long long s_idx, s_base;
  __shared__ uint32_t s_tail, s_epoch;
  __shared__ int s_hit;
  const int tid = threadIdx.x;
  const int lane = tid % kWave, wv = tid / kWave;
  const GraphView g = a.g;
  const int slot = blockIdx.x;
  uint32_t* stamp = a.big_stamp + (size_t)slot * (size_t)g.n;
  int32_t* queue = a.big_queue + (size_t)slot * (size_t)g.n;
  const unsigned long long ndef = deferred_count(a);
  Acc acc;

  for (;;) {
    if (tid == 0) {
      s_idx = atomicAdd(&a.ctr[kCtrNextBig], 1ull);
      s_epoch = a.big_epoch[slot] + 1u;
    }
    __syncthreads();
    const unsigned long long idx = s_idx;
    if (idx >= ndef) break;
    uint32_t epoch = s_epoch;
    if (epoch == 0u) {  // stamp counter wrapped: start the slot afresh
      for (int64_t i = tid; i < g.n; i += T) stamp[i] = 0u;
      epoch = 1u;
    }
    const unsigned long long rel = a.deferred[idx];
    const SetStream st = make_set_stream(a.seed, a.phase, a.first + rel);
    const int32_t root = draw_root(st, g.n);
    __syncthreads();
    if (tid == 0) {
      a.big_epoch[slot] = epoch;
      stamp[root] = epoch;
      queue[0] = root;
      s_tail = 1u;
      s_hit = (MODE == kModeCover && in_seed(a.seed_bits, root)) ? 1 : 0;
    }
    __syncthreads();
    int64_t head = 0;
    unsigned long long wloc = 0;
    for (;;) {
      const int64_t tail = (int64_t)s_tail;
      if (head >= tail || s_hit) break;
      const int nb = (int)min<int64_t>(tail - head, (int64_t)T);
      int64_t ea = 0, d = 0;
      uint32_t ng = 0;
      if (tid < nb) {
        const int32_t v = queue[head + tid];
        ea = g.off[v];
        const int64_t eb = g.off[v + 1];
        d = eb - ea;
        ng = d ? (uint32_t)(((eb - 1) >> 2) - (ea >> 2) + 1) : 0u;
      }
      wloc += (unsigned long long)d;
      uint32_t incl = wave_incl_scan(ng, lane);
      if (lane == kWave - 1) s_wtot[wv] = incl;
      __syncthreads();
      uint32_t carry = 0;
      for (int w = 0; w < wv; ++w) carry += s_wtot[w];
      incl += carry;
      s_incl[tid] = incl;
      s_ea[tid] = ea;
      s_d[tid] = d;
      __syncthreads();
      const uint32_t total = s_incl[T - 1];
      head += nb;
      for (uint32_t base = 0; base < total; base += T) {
        const uint32_t item = base + (uint32_t)tid;
        if (item < total) {
          int lo = 0, hi = nb - 1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_incl[mid] > item) hi = mid;
            else lo = mid + 1;
          }
          const int64_t oa = s_ea[lo], od = s_d[lo];
          const uint32_t oex = lo ? s_incl[lo - 1] : 0u;
          const int64_t grp = (oa >> 2) + (int64_t)(item - oex);
          const int4 s4 = reinterpret_cast<const int4*>(g.src)[grp];
          uint4 t4 = make_uint4(0u, 0u, 0u, 0u);
          if (!WC) t4 = reinterpret_cast<const uint4*>(g.thr)[grp];
          const uint4 x = draw(st, kKindCoin, (uint64_t)grp);
          const int32_t sv[4] = {s4.x, s4.y, s4.z, s4.w};
          const uint32_t xv[4] = {x.x, x.y, x.z, x.w};
          const uint32_t tv[4] = {t4.x, t4.y, t4.z, t4.w};
          const int64_t e0 = grp << 2;
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int64_t e = e0 + w;
            if (e < oa || e >= oa + od) continue;
            if (!edge_live<WC>(xv[w], tv[w], od)) continue;
            const int32_t u = sv[w];
            if (atomicExch(&stamp[u], epoch) != epoch) {
              const uint32_t pos = atomicAdd(&s_tail, 1u);
              queue[pos] = u;
              if (MODE == kModeCover && in_seed(a.seed_bits, u)) s_hit = 1;
            }
          }
        }
      }
      __syncthreads();
    }
    const unsigned long long wsum_w = wave_sum(wloc);
    if (lane == 0) s_red[wv] = wsum_w;
    __syncthreads();
    const uint32_t len = s_tail;
    if (MODE == kModeEmit) {
      if (tid == 0) {
        unsigned long long width = 0;
        for (int w = 0; w < T / kWave; ++w) width += s_red[w];
        const unsigned long long b = atomicAdd(&a.ctr[kCtrPoolCursor], (unsigned long long)len);
        s_base = b;
        a.set_start[rel] = b;
        a.set_len[rel] = len;
        if (a.widths) a.widths[rel] = width;
        acc.width += width;
        acc.nodes += len;
      }
      __syncthreads();
      const unsigned long long b = s_base;
      if (b + len <= a.pool_cap)
        for (uint32_t i = tid; i < len; i += T) a.pool[b + i] = queue[i];
    } else if (tid == 0) {
      unsigned long long width = 0;
      for (int w = 0; w < T / kWave; ++w) width += s_red[w];
      if (MODE == kModeWidth) {
        acc.kappa += kappa_fixed(width, g.m, a.k);
        acc.width += width;
        acc.nodes += len;
        if (a.widths) a.widths[rel] = width;
        if (a.sizes) a.sizes[rel] = len;
      } else if (s_hit) {
        acc.covered += 1;
      }
    }
    __syncthreads();
  }
  if (tid == 0) flush(a, acc);
}

// LT: one lane per set, visited stamps and chain in device memory.
template <int MODE>
__global__ __launch_bounds__(kWave) void lt_big_kernel(SampleArgs a) {
  const int slot = blockIdx.x * kWave + threadIdx.x;
  if (slot >= a.big_slots) return;
  const GraphView g = a.g;
  uint32_t* stamp = a.big_stamp + (size_t)slot * (size_t)g.n;
  int32_t* chain = a.big_queue + (size_t)slot * (size_t)g.n;
  const unsigned long long ndef = deferred_count(a);
  uint32_t epoch = a.big_epoch[slot];
  Acc acc;
  for (;;) {
    const unsigned long long idx = atomicAdd(&a.ctr[kCtrNextBig], 1ull);
    if (idx >= ndef) break;
    if (++epoch == 0u) {
      for (int64_t i = 0; i < g.n; ++i) stamp[i] = 0u;
      epoch = 1u;
    }
    const unsigned long long rel = a.deferred[idx];
    const SetStream st = make_set_stream(a.seed, a.phase, a.first + rel);
    int32_t v = draw_root(st, g.n);
    stamp[v] = epoch;
    chain[0] = v;
    int64_t len = 1;
    unsigned long long width = 0;
    bool hit = (MODE == kModeCover) && in_seed(a.seed_bits, v);
    while (!hit) {
      const int64_t ea = g.off[v];
      const int64_t d = g.off[v + 1] - ea;
      width += (unsigned long long)d;
      if (d == 0) break;
      const uint64_t j = scale64(draw(st, kKindPick, (uint64_t)v), (uint64_t)d);
      const int32_t u = g.src[ea + (int64_t)j];
      if (stamp[u] == epoch) break;
      stamp[u] = epoch;
      chain[len++] = u;
      v = u;
      if (MODE == kModeCover && in_seed(a.seed_bits, u)) hit = true;
    }
    if (MODE == kModeWidth) {
      acc.kappa += kappa_fixed(width, g.m, a.k);
      acc.width += width;
      acc.nodes += (unsigned long long)len;
      if (a.widths) a.widths[rel] = width;
      if (a.sizes) a.sizes[rel] = (uint32_t)len;
    } else if (MODE == kModeEmit) {
      const unsigned long long b = atomicAdd(&a.ctr[kCtrPoolCursor], (unsigned long long)len);
      if (b + (unsigned long long)len <= a.pool_cap)
        for (int64_t i = 0; i < len; ++i) a.pool[b + i] = chain[i];
      a.set_start[rel] = b;
      a.set_len[rel] = (uint32_t)len;
      if (a.widths) a.widths[rel] = width;
      acc.width += width;
      acc.nodes += (unsigned long long)len;
    } else if (hit) {
      acc.covered += 1;
    }
  }
  a.big_epoch[slot] = epoch;
  flush(a, acc);
}

__global__ void clear_counters_kernel(unsigned long long* ctr) {
  if (threadIdx.x < kCtrCount) ctr[threadIdx.x] = 0ull;
}

template <typename K>
int blocks_per_cu(K kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

}  // namespace

void launch_clear_counters(unsigned long long* ctr, hipStream_t s) {
  hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(64), 0, s, ctr);
}

int ic_wave_blocks_per_cu(int mode, bool wc) {
  switch (mode * 2 + (wc ? 1 : 0)) {
    case 0: return blocks_per_cu(ic_wave_kernel<kModeWidth, false>, kIcWaves * kWave);
    case 1: return blocks_per_cu(ic_wave_kernel<kModeWidth, true>, kIcWaves * kWave);
    case 2: return blocks_per_cu(ic_wave_kernel<kModeEmit, false>, kIcWaves * kWave);
    case 3: return blocks_per_cu(ic_wave_kernel<kModeEmit, true>, kIcWaves * kWave);
    case 4: return blocks_per_cu(ic_wave_kernel<kModeCover, false>, kIcWaves * kWave);
    default: return blocks_per_cu(ic_wave_kernel<kModeCover, true>, kIcWaves * kWave);
  }
}

int lt_lane_blocks_per_cu(int mode) {
  switch (mode) {
    case 0: return blocks_per_cu(lt_lane_kernel<kModeWidth>, kLtWaves * kWave);
    case 1: return blocks_per_cu(lt_lane_kernel<kModeEmit>, kLtWaves * kWave);
    default: return blocks_per_cu(lt_lane_kernel<kModeCover>, kLtWaves * kWave);
  }
}

void launch_sample(int model, int mode, const SampleArgs& a, int grid, hipStream_t s) {
  if (model == 0) {
    const dim3 blk(kIcWaves * kWave);
    const bool wc = a.g.thr == nullptr;
    switch (mode * 2 + (wc ? 1 : 0)) {
      case 0: hipLaunchKernelGGL((ic_wave_kernel<kModeWidth, false>), dim3(grid), blk, 0, s, a); break;
      case 1: hipLaunchKernelGGL((ic_wave_kernel<kModeWidth, true>), dim3(grid), blk, 0, s, a); break;
      case 2: hipLaunchKernelGGL((ic_wave_kernel<kModeEmit, false>), dim3(grid), blk, 0, s, a); break;
      case 3: hipLaunchKernelGGL((ic_wave_kernel<kModeEmit, true>), dim3(grid), blk, 0, s, a); break;
      case 4: hipLaunchKernelGGL((ic_wave_kernel<kModeCover, false>), dim3(grid), blk, 0, s, a); break;
      default: hipLaunchKernelGGL((ic_wave_kernel<kModeCover, true>), dim3(grid), blk, 0, s, a); break;
    }
  } else {
    const dim3 blk(kLtWaves * kWave);
    switch (mode) {
      case 0: hipLaunchKernelGGL((lt_lane_kernel<kModeWidth>), dim3(grid), blk, 0, s, a); break;
      case 1: hipLaunchKernelGGL((lt_lane_kernel<kModeEmit>), dim3(grid), blk, 0, s, a); break;
      default: hipLaunchKernelGGL((lt_lane_kernel<kModeCover>), dim3(grid), blk, 0, s, a); break;
    }
  }
}

void launch_sample_large(int model, int mode, const SampleArgs& a, hipStream_t s) {
  if (model == 0) {
    const dim3 grid(a.big_slots), blk(kBigThreads);
    const bool wc = a.g.thr == nullptr;
    switch (mode * 2 + (wc ? 1 : 0)) {
      case 0: hipLaunchKernelGGL((ic_big_kernel<kModeWidth, false>), grid, blk, 0, s, a); break;
      case 1: hipLaunchKernelGGL((ic_big_kernel<kModeWidth, true>), grid, blk, 0, s, a); break;
      case 2: hipLaunchKernelGGL((ic_big_kernel<kModeEmit, false>), grid, blk, 0, s, a); break;
      case 3: hipLaunchKernelGGL((ic_big_kernel<kModeEmit, true>), grid, blk, 0, s, a); break;
      case 4: hipLaunchKernelGGL((ic_big_kernel<kModeCover, false>), grid, blk, 0, s, a); break;
      default: hipLaunchKernelGGL((ic_big_kernel<kModeCover, true>), grid, blk, 0, s, a); break;
    }
  } else {
    const dim3 grid((a.big_slots + kWave - 1) / kWave), blk(kWave);
    switch (mode) {
      case 0: hipLaunchKernelGGL((lt_big_kernel<kModeWidth>), grid, blk, 0, s, a); break;
      case 1: hipLaunchKernelGGL((lt_big_kernel<kModeEmit>), grid, blk, 0, s, a); break;
      default: hipLaunchKernelGGL((lt_big_kernel<kModeCover>), grid, blk, 0, s, a); break;
    }
  }
}

}  // namespace tim
