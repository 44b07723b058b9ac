// RR-set samplers for gfx950 (Definitions 1-2; Section 3.1; Section 4.2).
//
// IC (reverse BFS over in-edges), tier 0: a wavefront is split into segments
// of S lanes and every segment builds its own RR set, so one wavefront keeps
// 64/S sets in flight and their memory latencies overlap.  A set's nodes live
// in an LDS queue (which is also its output list); visited nodes are found
// through an LDS membership signature (segments of up to 8 lanes) or an LDS
// open-addressing hash (wider ones).  Each iteration of the loop, every segment either
// loads its next batch of up to S queued nodes (two CSR offsets per lane, a
// segmented prefix sum of their 4-edge groups) or processes S groups of the
// current batch: a lane loads 4 consecutive sources with one 16-byte load,
// draws one Philox block for the group and decides the 4 edges with its 4
// words; live edges into unvisited nodes are appended to the queue.  Sets
// that outgrow the segment's LDS structures are deferred: a set is a pure
// function of its keys, so restarting it in another tier gives the same set.
// Tier 1 is the same kernel with one set per wavefront and 8x the LDS
// capacity; the last tier is a 512-thread block per set with visited stamps
// and a queue of n entries in device memory.
//
// General triggering (Section 4.2): one set per wavefront over an LDS queue
// and hash; larger sets go to a block per set with device-memory stamps.
//
// LT (at most one live in-edge per node): each lane walks one set's chain,
// kept in LDS with a 256-bit membership signature in registers; longer chains
// go to the last tier, one lane per chain without visited marks (Brent's
// cycle search over the walk, which is a fixed function of the set's keys).
//
// Every launch also reduces what the phase needs: the widths (Equation (1)),
// the set sizes, the number of sets meeting a seed set (Algorithm 3, RefineKPT's test)
// and, in width mode, the exact 128-bit sum of kappa(R) * 2^53 (Equation (8)),
// computed by a separate pass over the widths so that the binary64 kappa
// arithmetic runs one set per lane instead of inside the traversal loop.
#include <stdlib.h>

#include "engine.hpp"
#include "pick.hpp"
#include "rng.hpp"

namespace tim {
namespace {

constexpr int kWave = 64;
constexpr int kSegThreads = 256;   // block size of the IC segment kernels
constexpr int kLtWaves = 2;        // wavefronts per block, LT lane-level pass
constexpr int kChain = 64;         // LT chain length held in LDS
constexpr int kBigThreads = 512;   // IC last-tier block size
constexpr int kSegGroups = 1;      // 4-edge groups a lane decides per step (IC tiers 0 and 1)
constexpr int kSegPasses = 2;      // batches of queued nodes a segment may take per iteration (IC tiers 0 and 1)
constexpr uint64_t kKappaBlocks = 1024;  // largest grid of the kappa pass (four per CU)

typedef unsigned __int128 u128;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane 0's value in every lane, as a wave-uniform (scalar-register) value:
// device-atomic results that lane 0 fetched for the whole wavefront.  Through
// __shfl the compiler keeps them, and what is derived from them, in vector
// registers.
__device__ __forceinline__ unsigned long long lane0_u64(unsigned long long x) {
  return ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(x >> 32)) << 32) |
         (unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)x);
}

// x from the lane O below in the same 16-lane DPP row (0 where that leaves the row).
template <int O>
__device__ __forceinline__ uint32_t dpp_row_shr(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x110 + O, 0xF, 0xF, true);
}

// Inclusive prefix sum within segments of W lanes.  Segments of up to 16
// lanes lie inside one DPP row, so their steps are row shifts (no LDS
// crossbar); lanes closer than the shift to their segment's start add nothing.
// The shifted value is taken in every lane before the select: a DPP move
// under a narrowed exec mask would read 0 from the disabled lanes below.
template <int W>
__device__ __forceinline__ uint32_t seg_incl_scan(uint32_t x, int sl) {
  if constexpr (W <= 16) {
    uint32_t y;
    if constexpr (W > 1) { y = dpp_row_shr<1>(x); x += sl >= 1 ? y : 0u; }
    if constexpr (W > 2) { y = dpp_row_shr<2>(x); x += sl >= 2 ? y : 0u; }
    if constexpr (W > 4) { y = dpp_row_shr<4>(x); x += sl >= 4 ? y : 0u; }
    if constexpr (W > 8) { y = dpp_row_shr<8>(x); x += sl >= 8 ? y : 0u; }
    return x;
  } else if constexpr (W == 64) {
    // whole wavefront (every lane active): scan each 16-lane row, then add
    // row 0's total to rows 1 and 3 and rows 0-1's total to rows 2 and 3
    x += dpp_row_shr<1>(x);
    x += dpp_row_shr<2>(x);
    x += dpp_row_shr<4>(x);
    x += dpp_row_shr<8>(x);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
  } else {
#pragma unroll
    for (int o = 1; o < W; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, W);
      if (sl >= o) x += y;
    }
    return x;
  }
}

// Sum over segments of W lanes, in every lane of the segment.  Up to 16
// lanes: a butterfly of DPP moves (swap neighbours, swap pairs in a quad,
// then mirror the 8-lane and 16-lane halves), each step adding two disjoint
// partial sums.
template <int W>
__device__ __forceinline__ uint32_t seg_sum_u32(uint32_t x) {
  if constexpr (W <= 16) {
    if constexpr (W > 1) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
    if constexpr (W > 2) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
    if constexpr (W > 4) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false);  // half mirror
    if constexpr (W > 8) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false);  // mirror
    return x;
  } else {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, W);
    return x;
  }
}

// A segment's total in every lane of it, given the inclusive scan `incl` of
// the values `x`: a DPP sum up to 16 lanes, the last lane read out for the
// whole wavefront, else a shuffle from the segment's last lane.
template <int W>
__device__ __forceinline__ uint32_t seg_last(uint32_t incl, uint32_t x) {
  if constexpr (W <= 16) return seg_sum_u32<W>(x);
  else if constexpr (W == 64) return (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
  else return __shfl(incl, W - 1, W);
}

template <int W>
__device__ __forceinline__ unsigned long long seg_sum(unsigned long long x) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, W);
  return x;
}

// The W bits of a 64-lane ballot that belong to segment sw.
template <int W>
__device__ __forceinline__ uint64_t seg_bits(uint64_t m, int sw) {
  if (W == 64) return m;
  return (m >> (sw * W)) & ((1ull << (W & 63)) - 1ull);
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

// Open addressing in LDS over 2^HLOG slots, key u+1 (0 = empty).
// Returns 1: inserted, 0: already present, -1: table full.
template <int HLOG>
__device__ __forceinline__ int lds_insert(uint32_t* h, uint32_t u) {
  constexpr uint32_t H = 1u << HLOG;
  const uint32_t key = u + 1u;
  uint32_t pos = (u * 0x9E3779B1u) >> (32 - HLOG);
  for (uint32_t i = 0; i < H; ++i) {
    const uint32_t cur = h[pos];
    if (cur == key) return 0;
    if (cur == 0u) {
      const uint32_t old = atomicCAS(&h[pos], 0u, key);
      if (old == 0u) return 1;
      if (old == key) return 0;
    }
    pos = (pos + 1u) & (H - 1u);
  }
  return -1;
}

// One bit of a 64-bit membership signature: a clear bit proves absence.
__device__ __forceinline__ uint64_t sig_bit(int32_t u) { return 1ull << (((uint32_t)u * 0x9E3779B1u) >> 26); }

// A 256-bit membership signature in four registers (a clear bit proves
// absence); the word is chosen by selects, so the array never leaves registers.
struct Sig256 {
  uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
  __device__ __forceinline__ static uint32_t hash(int32_t u) { return (uint32_t)u * 0x9E3779B1u; }
  __device__ __forceinline__ bool maybe(int32_t u) const {
    const uint32_t h = hash(u), wd = h >> 30;
    const uint64_t w = wd == 0u ? w0 : wd == 1u ? w1 : wd == 2u ? w2 : w3;
    return (w >> ((h >> 24) & 63u)) & 1ull;
  }
  __device__ __forceinline__ void add(int32_t u) {
    const uint32_t h = hash(u), wd = h >> 30;
    const uint64_t b = 1ull << ((h >> 24) & 63u);
    w0 |= wd == 0u ? b : 0ull;
    w1 |= wd == 1u ? b : 0ull;
    w2 |= wd == 2u ? b : 0ull;
    w3 |= wd == 3u ? b : 0ull;
  }
};
// A set signature of kSigWords 32-bit words (1024 bits): word index and bit
// of node u.  The top bits of a multiplicative hash pick the word, the 5 bits
// below them the bit.
constexpr int kSigWordBits = 5;
constexpr int kSigWords = 1 << kSigWordBits;
__device__ __forceinline__ uint32_t sig_hash(int32_t u) { return (uint32_t)u * 0x9E3779B1u; }
__device__ __forceinline__ uint32_t sig_word(uint32_t h) { return h >> (32 - kSigWordBits); }
__device__ __forceinline__ uint32_t sig_bit(uint32_t h) { return 1u << ((h >> (27 - kSigWordBits)) & 31u); }

struct Acc {
  u128 kappa = 0;
  unsigned long long width = 0, nodes = 0, covered = 0;
};

// Places a wavefront's sets finished in one step in its node-pool slice
// [pool_next, pool_end).  `mine` is this lane's entry count (0 if none),
// `winc` its inclusive prefix over the wavefront and `tot` the total.  The
// sets whose prefix fits the slice go there; the rest go to a new slice of
// max(slice, rest) entries, so what is left unused of the old slice is
// shorter than the first set that did not fit.  Returns this lane's offset.
__device__ __forceinline__ unsigned long long pool_place(const SampleArgs& a, unsigned long long slice, uint32_t mine,
                                                         uint32_t winc, uint32_t tot, unsigned long long& pool_next,
                                                         unsigned long long& pool_end, int lane) {
  const unsigned long long room = pool_end - pool_next;
  const bool fits = (unsigned long long)winc <= room;
  const uint64_t fm = __ballot(fits);  // a prefix of the lanes: winc grows with the lane
  const int nfit = __popcll(fm);
  const uint32_t used = nfit ? (uint32_t)__builtin_amdgcn_readlane((int)winc, nfit - 1) : 0u;
  unsigned long long pos = pool_next + (unsigned long long)(winc - mine);
  if (used == tot) {
    pool_next += tot;
    return pos;
  }
  const unsigned long long rest = (unsigned long long)(tot - used);
  const unsigned long long want = max(slice, rest);
  unsigned long long got = 0;
  if (lane == 0) got = atomicAdd(&a.ctr[kCtrPoolCursor], want);
  got = lane0_u64(got);
  if (!fits) pos = got + (unsigned long long)(winc - mine - used);
  pool_next = got + rest;
  pool_end = got + want;
  return pos;
}

// Sum of every lane's accumulators, added to the counters by lane 0.
__device__ __forceinline__ void wave_flush(const SampleArgs& a, const Acc& acc, int tier, int lane) {
  const unsigned long long lo = (unsigned long long)acc.kappa, hi = (unsigned long long)(acc.kappa >> 64);
  const unsigned long long s_hi = seg_sum<kWave>(hi);
  const unsigned long long s_l0 = seg_sum<kWave>(lo & 0xFFFFFFFFull);
  const unsigned long long s_l1 = seg_sum<kWave>(lo >> 32);
  const unsigned long long w = seg_sum<kWave>(acc.width);
  const unsigned long long nd = seg_sum<kWave>(acc.nodes);
  const unsigned long long cv = seg_sum<kWave>(acc.covered);
  if (lane == 0) {
    unsigned long long* c = a.ctr + kCtrAcc + kAccStride * tier;
    add_u128(c + kAccKappaLo, ((u128)s_hi << 64) + ((u128)s_l1 << 32) + (u128)s_l0);
    if (w) atomicAdd(c + kAccWidth, w);
    if (nd) atomicAdd(c + kAccNodes, nd);
    if (cv) atomicAdd(c + kAccCovered, cv);
  }
}

// A block's accumulators in LDS.  Every wavefront adds its sums here when
// it is done; the last one of the block adds the total to the counters, so
// a launch makes one set of device atomics per block instead of one per
// wavefront (atomics on one address serialize).  Wavefronts that leave
// early count themselves done too.  Batched launches flush per wavefront:
// the wavefronts of a block may be working for different jobs.
struct BlockAcc {
  unsigned long long v[6];  // kappa high word, kappa low word's two halves, width, nodes, covered
  unsigned int done;
};

__device__ __forceinline__ void block_acc_init(BlockAcc& b) {
  if (threadIdx.x < 6) b.v[threadIdx.x] = 0ull;
  if (threadIdx.x == 0) b.done = 0u;
  __syncthreads();
}

__device__ __forceinline__ void block_acc_flush(const SampleArgs& a, BlockAcc& b, const Acc& acc, int tier,
                                                int lane) {
  const unsigned long long lo = (unsigned long long)acc.kappa, hi = (unsigned long long)(acc.kappa >> 64);
  unsigned long long s[6];
  s[0] = seg_sum<kWave>(hi);
  s[1] = seg_sum<kWave>(lo >> 32);
  s[2] = seg_sum<kWave>(lo & 0xFFFFFFFFull);
  s[3] = seg_sum<kWave>(acc.width);
  s[4] = seg_sum<kWave>(acc.nodes);
  s[5] = seg_sum<kWave>(acc.covered);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i)
      if (s[i]) __hip_atomic_fetch_add(&b.v[i], s[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const unsigned int nw = blockDim.x / kWave;
    if (__hip_atomic_fetch_add(&b.done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == nw - 1u) {
      unsigned long long t[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) t[i] = __hip_atomic_load(&b.v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      unsigned long long* c = a.ctr + kCtrAcc + kAccStride * tier;
      // per-wavefront limbs are below 2^39, so 64-bit block sums of them are exact
      add_u128(c + kAccKappaLo, ((u128)t[0] << 64) + ((u128)t[1] << 32) + (u128)t[2]);
      if (t[3]) atomicAdd(c + kAccWidth, t[3]);
      if (t[4]) atomicAdd(c + kAccNodes, t[4]);
      if (t[5]) atomicAdd(c + kAccCovered, t[5]);
    }
  }
}

// Flush through the block when it has a BlockAcc, else per wavefront.
__device__ __forceinline__ void flush_acc(const SampleArgs& a, BlockAcc* b, const Acc& acc, int tier, int lane) {
  if (b) block_acc_flush(a, *b, acc, tier, lane);
  else wave_flush(a, acc, tier, lane);
}

__device__ __forceinline__ void block_flush(const SampleArgs& a, const Acc& acc, int tier) {
  unsigned long long* c = a.ctr + kCtrAcc + kAccStride * tier;
  add_u128(c + kAccKappaLo, acc.kappa);
  if (acc.width) atomicAdd(c + kAccWidth, acc.width);
  if (acc.nodes) atomicAdd(c + kAccNodes, acc.nodes);
  if (acc.covered) atomicAdd(c + kAccCovered, acc.covered);
}

__device__ __forceinline__ unsigned long long list_len(const SampleArgs& a, int ctr) {
  const unsigned long long d = a.ctr[ctr];
  return d < a.count ? d : a.count;
}

// Wave-uniform reservoir of work items [cur, end), refilled `chunk` at a time.
struct Reservoir {
  unsigned long long cur = 0, end = 0, chunk = 1;
  int part = 0, tried = 0;  // the part of the range being taken, and parts found spent
};

// Items per refill: about 4 refills per wavefront over the launch (each is a
// device atomic on a work cursor, and those on one cursor serialize), at
// least one item per requester, at most 64 per requester.
__device__ __forceinline__ unsigned long long chunk_for(unsigned long long total, int waves_per_block,
                                                        int per_wave) {
  const unsigned long long waves = (unsigned long long)gridDim.x * (unsigned long long)waves_per_block;
  unsigned long long c = total / (waves * 4ull);
  c = c < (unsigned long long)per_wave ? (unsigned long long)per_wave : c;
  return c > 64ull * per_wave ? 64ull * per_wave : c;
}

// Refills a wavefront's reservoir from its part of [0, total).  SPLIT: the
// range is split into kCtrParts parts (a power of two, so the bounds are
// shifts) with a cursor each, kCtrPartStride words apart from next_ctr, and a
// spent part sends the wavefront on to the next one; else one cursor at
// next_ctr.  False once every part is spent.  Cursor values and the part
// reach the wavefront through readfirstlane, which keeps the reservoir in
// scalar registers (with __shfl they took vector registers, and the stored-
// set kernel fell from 6 to 5 wavefronts per SIMD).
template <bool SPLIT>
__device__ __forceinline__ bool refill_parts(const SampleArgs& a, int next_ctr, unsigned long long total, Reservoir& r,
                                             int lane) {
  constexpr int np = SPLIT ? (int)kCtrParts : 1;
  r.part = __builtin_amdgcn_readfirstlane(r.part);
  r.tried = __builtin_amdgcn_readfirstlane(r.tried);
  while (r.tried < np) {
    const unsigned long long pb = SPLIT ? total * (unsigned long long)r.part / kCtrParts : 0ull;
    const unsigned long long pe = SPLIT ? total * (unsigned long long)(r.part + 1) / kCtrParts : total;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&a.ctr[next_ctr + kCtrPartStride * r.part], r.chunk);
    base = lane0_u64(base);
    if (pb + base < pe) {
      r.cur = pb + base;
      r.end = min(pb + base + r.chunk, pe);
      return true;
    }
    r.tried += 1;
    r.part = r.part + 1 == np ? 0 : r.part + 1;
  }
  return false;
}

// refill_parts for a part count given at run time (TierIO::parts: 0, 1 or kCtrParts).
__device__ __forceinline__ bool refill(const SampleArgs& a, int next_ctr, int parts, unsigned long long total,
                                       Reservoir& r, int lane) {
  return parts > 1 ? refill_parts<true>(a, next_ctr, total, r, lane) : refill_parts<false>(a, next_ctr, total, r, lane);
}

// Hands one work item to every requester (lanes with want && is_leader); all
// lanes of a segment see their leader's result through below_leader.  Lanes
// that get nothing because the work is gone set exhausted.
__device__ __forceinline__ bool take(const SampleArgs& a, int next_ctr, int parts, unsigned long long total,
                                     Reservoir& r, bool want, bool is_leader, uint64_t below_leader, int lane,
                                     bool& exhausted, unsigned long long& item) {
  bool got = false;
  uint64_t wmask = __ballot(want && is_leader);
  while (wmask) {
    if (r.cur >= r.end && !refill(a, next_ctr, parts, total, r, lane)) {
      if (want) exhausted = true;
      break;
    }
    const unsigned long long avail = r.end - r.cur;
    const unsigned long long rank = (unsigned long long)__popcll(wmask & below_leader);
    if (want && rank < avail) {
      item = r.cur + rank;
      got = true;
      want = false;
    }
    const unsigned long long nw = (unsigned long long)__popcll(wmask);
    r.cur += nw < avail ? nw : avail;
    wmask = __ballot(want && is_leader);
  }
  return got;
}

// Roots of the sets a wavefront hands out, drawn 64 at a time: lane j holds
// the root (and set id) of reservoir item base + j, so one Philox call per lane
// serves 64 sets instead of one call per set issued across the wavefront.
struct RootBuffer {
  unsigned long long base = ~0ull;
  unsigned long long rel = 0;  // lane j: relative set id of item base + j
  int32_t root = 0;            // lane j: its root
};

__device__ __forceinline__ void fill_roots(const SampleArgs& a, const TierIO& io, unsigned long long total,
                                           unsigned long long base, RootBuffer& rb, int lane) {
  rb.base = base;
  const unsigned long long item = base + (unsigned long long)lane;
  if (item < total) {
    rb.rel = io.in_list ? io.in_list[item] : item;
    rb.root = draw_root(make_key(a.seed), make_set_stream(a.phase, a.first + rb.rel), a.g.n);
  }
}

// take() for the IC kernels: hands one item to every requesting segment and
// returns its set id and root from the wavefront's root buffer.
template <bool SPLIT>
__device__ __forceinline__ bool take_set(const SampleArgs& a, const TierIO& io, unsigned long long total, Reservoir& r,
                                         RootBuffer& rb, bool want, bool is_leader, uint64_t below_leader, int lane,
                                         bool& exhausted, unsigned long long& rel, int32_t& root) {
  bool got = false;
  unsigned long long item = 0;
  uint64_t wmask = __ballot(want && is_leader);
  while (wmask) {
    if (r.cur >= r.end && !refill_parts<SPLIT>(a, io.next_ctr, total, r, lane)) {
      if (want) exhausted = true;
      break;
    }
    const unsigned long long avail = r.end - r.cur;
    const unsigned long long nw = (unsigned long long)__popcll(wmask);
    const unsigned long long give = nw < avail ? nw : avail;
    if (r.cur < rb.base || r.cur + give > rb.base + (unsigned long long)kWave) fill_roots(a, io, total, r.cur, rb, lane);
    const unsigned long long rank = (unsigned long long)__popcll(wmask & below_leader);
    const bool mine = want && rank < avail;
    const int src = (int)(r.cur + rank - rb.base) & (kWave - 1);
    const unsigned long long rel_x = __shfl(rb.rel, src);
    const int32_t root_x = __shfl(rb.root, src);
    if (mine) {
      item = r.cur + rank;
      rel = rel_x;
      root = root_x;
      got = true;
      want = false;
    }
    r.cur += give;
    wmask = __ballot(want && is_leader);
  }
  (void)item;
  return got;
}

// ------------------------------------------------------------------------
// IC, tiers 0 and 1: S lanes per set.  Edge positions fit 32 bits (m < 2^32).
// HLOG > 0: visited nodes are marked in an LDS hash of 2^HLOG slots and live
// edges are inserted concurrently.  HLOG == 0: no hash, which leaves the LDS
// to more sets in flight; a 1024-bit LDS signature per set proves most
// sources new (an atomic OR settles sources sharing a bit), and the rest are
// looked up one at a time in the set's own queue (each of the S lanes scans
// Q/S entries).
// Width mode writes w(R) per set; kappa is summed by kappa_reduce_kernel.
// ------------------------------------------------------------------------
// first_only: a launch of its own over one deferred list, whose wavefronts
// beyond the first ones the list needs leave at once instead of each taking
// a turn at the list's cursor.
template <int MODE, bool WC, int S, int Q, int HLOG, int GMAX, int R, bool SPLIT = false>
__device__ __forceinline__ void ic_seg_run(const SampleArgs& a, const TierIO& io, bool first_only,
                                           BlockAcc* blk = nullptr) {
  constexpr bool kHash = HLOG > 0;
  constexpr int H = kHash ? (1 << HLOG) : 4;
  constexpr int NSEG = kSegThreads / S;
  __shared__ int32_t s_q[NSEG][Q];
  __shared__ uint32_t s_h[kHash ? NSEG : 1][H];
  __shared__ uint32_t s_tail[kHash ? NSEG : 1];
  __shared__ __align__(16) uint32_t s_sig[kHash ? 1 : NSEG][kSigWords];  // signature of each set's queued nodes
  const int lane = threadIdx.x % kWave;
  const int sl = threadIdx.x % S;       // lane within the segment
  const int seg = threadIdx.x / S;      // segment within the block
  const int sw = lane / S;              // segment within the wavefront
  const int leader = sw * S;            // wavefront lane of the segment's first lane
  const bool is_leader = sl == 0;
  const uint64_t below_leader = leader ? (~0ull >> (64 - leader)) : 0ull;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  int32_t* q = s_q[seg];
  uint32_t* h = s_h[kHash ? seg : 0];
  const GraphView g = a.g;
  const Key key = make_key(a.seed);
  const unsigned long long total = io.in_list ? list_len(a, io.in_len_ctr) : a.count;
  if (first_only && io.in_list) {
    const unsigned long long wave = (unsigned long long)blockIdx.x * (kSegThreads / kWave) + threadIdx.x / kWave;
    if (wave * (unsigned long long)(kWave / S) >= total) {
      flush_acc(a, blk, Acc(), io.acc, lane);
      return;
    }
  }
  Acc acc;
  Reservoir res;
  res.chunk = chunk_for(total, kSegThreads / kWave, kWave / S);
  if (SPLIT) res.part = (int)(blockIdx.x % (unsigned)kCtrParts);  // blocks take turns over the XCDs
  RootBuffer rb;
  unsigned long long pool_next = 0, pool_end = 0;  // wavefront's slice of the node pool

  // segment state (the same in every lane of a segment)
  bool has = false, exhausted = false, hit = false, bad = false;
  unsigned long long rel = 0;
  SetStream st = make_set_stream(a.phase, a.first);
  int head = 0, tail_r = 0;                  // queue cursor; queue length (hash-free variant)
  uint32_t G = 0, done_items = 0, gsum = 0;  // groups of the current batch / done / of the set so far
  // lane state: this lane's node of the current batch
  uint32_t ea = 0, d = 0, ng = 0, incl = 0;
  uint32_t wlane = 0;

  for (;;) {
    // ---- A: segments whose set is complete finish it (or defer it), so that
    // they take their next set in this same iteration
    bool fin = false, defer_now = false;
    uint32_t fin_len = 0, fin_width = 0;
    if (has && (done_items >= G || hit || bad)) {
      const int tail = kHash ? (int)s_tail[seg] : tail_r;
      if (bad || tail > Q || hit || head >= tail) {
        fin_width = seg_sum_u32<S>(wlane);
        has = false;
        if (bad || tail > Q) {
          defer_now = true;
        } else {
          fin = true;
          fin_len = (uint32_t)tail;
          if (is_leader) {
            if (MODE == kModeWidth) {
              a.wbuf[rel] = fin_width;
              acc.width += fin_width;
              acc.nodes += fin_len;
              if (a.sizes) a.sizes[rel] = fin_len;
            } else if (MODE == kModeCover) {
              acc.width += fin_width;
              acc.nodes += fin_len;
              if (hit) acc.covered += 1;
            }
          }
        }
      }
    }

    // deferred sets go to the next tier's list, one atomic per wavefront
    {
      const bool dl = defer_now && is_leader;
      const uint64_t dm = __ballot(dl);
      if (dm) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&a.ctr[io.out_len_ctr], (unsigned long long)__popcll(dm));
        base = lane0_u64(base);
        if (dl) {
          const unsigned long long pos = base + (unsigned long long)__popcll(dm & below);
          if (pos < a.count) io.out_list[pos] = rel;
        }
      }
    }

    // stored sets: one reservation in the wavefront's pool slice per iteration
    if (MODE == kModeEmit) {
      const uint32_t mine = (fin && is_leader) ? fin_len : 0u;
      const uint64_t fm = __ballot(mine != 0u);
      if (fm) {
        const uint32_t winc = seg_incl_scan<kWave>(mine, lane);
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)winc, kWave - 1);
        // tier 0 reserves slices; the deferral tier (large sets, few) exactly what it stores
        const unsigned long long slice = io.acc == 0 ? (unsigned long long)a.pool_chunk : 0ull;
        const unsigned long long my_base = pool_place(a, slice, mine, winc, tot, pool_next, pool_end, lane);
        const unsigned long long base = __shfl(my_base, leader);
        if (fin) {
          if (base + fin_len <= a.pool_cap)
            for (uint32_t i = sl; i < fin_len; i += S) a.pool[base + i] = q[i];
          if (is_leader) {
            a.set_start[rel] = a.pool_base + base;
            a.set_len[rel] = fin_len;
            if (a.widths) a.widths[rel] = fin_width;
            if (a.wbuf) a.wbuf[rel] = fin_width;
            acc.width += fin_width;
            acc.nodes += fin_len;
          }
        }
      }
    }
    wave_sync();

    // ---- B: idle segments take their next set
    {
      int32_t root = 0;
      const bool want = !has && !exhausted;
      if (take_set<SPLIT>(a, io, total, res, rb, want, is_leader, below_leader, lane, exhausted, rel, root)) {
        st = make_set_stream(a.phase, a.first + rel);
        if (kHash) {
          uint4* h4 = reinterpret_cast<uint4*>(h);
          for (int i = sl; i < H / 4; i += S) h4[i] = make_uint4(0u, 0u, 0u, 0u);
          wave_sync();
        }
        if (is_leader) {
          q[0] = root;
          if (kHash) {
            s_tail[seg] = 1u;
            lds_insert<(kHash ? HLOG : 1)>(h, (uint32_t)root);
          }
        }
        tail_r = 1;
        if (!kHash) {  // the segment's lanes clear the words (the root is the same in all of them)
          const uint32_t hr = sig_hash(root), wd = sig_word(hr), bt = sig_bit(hr);
          uint4* s4 = reinterpret_cast<uint4*>(s_sig[seg]);
          for (int i = sl; i < kSigWords / 4; i += S) {
            const uint32_t w0 = 4u * (uint32_t)i;
            s4[i] = make_uint4(wd == w0 ? bt : 0u, wd == w0 + 1u ? bt : 0u, wd == w0 + 2u ? bt : 0u,
                               wd == w0 + 3u ? bt : 0u);
          }
        }
        has = true;
        hit = (MODE == kModeCover) && in_seed(a.seed_bits, root);
        bad = false;
        head = 0;
        G = 0;
        done_items = 0;
        gsum = 0;
        wlane = 0;
      }
    }
    if (__ballot(has) == 0) break;
    wave_sync();

    // C and D run up to kSegPasses times per iteration, so that the sets'
    // finishing and taking above are paid once per two batches; a second pass
    // runs only while some segment still has groups or queued nodes.
    for (int pass = 0; pass < kSegPasses; ++pass) {
      if (pass > 0) {
        const int tl = kHash ? (int)s_tail[seg] : tail_r;
        if (__ballot(has && !hit && !bad && (done_items < G || head < tl)) == 0ull) break;
      }

      // ---- C: segments whose batch is done load the next batch of queued nodes
      // (a set still held here that is not complete has queued nodes left)
      if (has && done_items >= G && !hit && !bad) {
        const int tail = kHash ? (int)s_tail[seg] : tail_r;
        const int nb = min(tail - head, S);
        ea = 0;
        d = 0;
        ng = 0;
        if (sl < nb) {
          const int32_t v = q[head + sl];
          ea = g.off32[v];  // with off32[v + 1]: one 8-byte load
          const uint32_t eb = g.off32[v + 1];
          d = eb - ea;
          ng = d ? ((eb - 1u) >> 2) - (ea >> 2) + 1u : 0u;
        }
        wlane += d;
        head += nb;
        incl = seg_incl_scan<S>(ng, sl);
        G = seg_last<S>(incl, ng);
        done_items = 0;
        gsum += G;
        if (gsum > (uint32_t)GMAX) {  // too wide for this tier: hand it on
          bad = true;
          done_items = G;
        }
      }

      // ---- D: segments with work process R*S groups of their batch (R per lane)
      bool lhit = false, lbad = false;
      if (has && done_items < G) {
        int32_t sv[4 * R];
        bool live[4 * R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t item = done_items + (uint32_t)(r * S + sl);
          int owner = 0;
#pragma unroll
          for (int step = S / 2; step > 0; step >>= 1) {
            const uint32_t c = __shfl(incl, owner + step - 1, S);
            if (c <= item) owner += step;
          }
          owner = min(owner, S - 1);
          const uint32_t oa = __shfl(ea, owner, S);
          const uint32_t od = __shfl(d, owner, S);
          const uint32_t oex = __shfl(incl - ng, owner, S);
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            sv[4 * r + w] = 0;
            live[4 * r + w] = false;
          }
          if (item < G) {
            const uint32_t grp = (oa >> 2) + (item - oex);
            const int4 s4 = reinterpret_cast<const int4*>(g.src)[grp];
            uint4 t4 = make_uint4(0u, 0u, 0u, 0u);
            if (!WC) t4 = reinterpret_cast<const uint4*>(g.thr)[grp];
            const uint4 x = draw(key, st, kKindCoin, (uint64_t)grp);
            sv[4 * r + 0] = s4.x;
            sv[4 * r + 1] = s4.y;
            sv[4 * r + 2] = s4.z;
            sv[4 * r + 3] = s4.w;
            const uint32_t xv[4] = {x.x, x.y, x.z, x.w};
            const uint32_t tv[4] = {t4.x, t4.y, t4.z, t4.w};
            const uint32_t e0 = grp << 2;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
              const uint32_t e = e0 + (uint32_t)w;
              live[4 * r + w] = e - oa < od && edge_live<WC>(xv[w], tv[w], od);
            }
          }
        }
        bool any_live = false;
#pragma unroll
        for (int w = 0; w < 4 * R; ++w) any_live |= live[w];
        if (kHash) {
#pragma unroll
          for (int w = 0; w < 4 * R; ++w) {
            if (!live[w]) continue;
            const int32_t u = sv[w];
            const int r = lds_insert<(kHash ? HLOG : 1)>(h, (uint32_t)u);
            if (r < 0) {
              lbad = true;
            } else if (r == 1) {
              const uint32_t pos = atomicAdd(&s_tail[seg], 1u);
              if (pos < (uint32_t)Q) q[pos] = u;
              else lbad = true;
              if (MODE == kModeCover && in_seed(a.seed_bits, u)) lhit = true;
            }
          }
        } else if (seg_bits<S>(__ballot(any_live), sw) != 0ull) {
          // Every live source sets its signature bit in the set's LDS signature
          // with an atomic OR.  One that finds the bit clear is new (every queued
          // node's bit is set, and of several sources sharing a bit in this step
          // only the first sees it clear): those are appended at once.  The rest
          // are looked up in the queue one at a time, after the appends.
          bool fast[4 * R];
          uint32_t nfast = 0;
#pragma unroll
          for (int w = 0; w < 4 * R; ++w) {
            fast[w] = false;
            if (live[w]) {
              const uint32_t hv = sig_hash(sv[w]), b = sig_bit(hv);
              fast[w] = (atomicOr(&s_sig[seg][sig_word(hv)], b) & b) == 0u;
            }
            nfast += fast[w] ? 1u : 0u;
          }
          const uint32_t fincl = seg_incl_scan<S>(nfast, sl);
          const uint32_t ftot = seg_last<S>(fincl, nfast);
          if (tail_r + (int)ftot > Q) {
            lbad = true;
          } else {
            int pos = tail_r + (int)(fincl - nfast);
#pragma unroll
            for (int w = 0; w < 4 * R; ++w) {
              if (!fast[w]) continue;
              q[pos++] = sv[w];
              if (MODE == kModeCover && in_seed(a.seed_bits, sv[w])) lhit = true;
            }
            tail_r += (int)ftot;
            wave_sync();
#pragma unroll
            for (int w = 0; w < 4 * R; ++w) {
              uint64_t m = seg_bits<S>(__ballot(live[w] && !fast[w]), sw);
              while (m) {
                const int src_lane = __ffsll((unsigned long long)m) - 1;
                m &= m - 1ull;
                const int32_t u = __shfl(sv[w], src_lane, S);
                bool found = false;
                for (int i = sl; i < tail_r; i += S) found |= q[i] == u;
                if (seg_bits<S>(__ballot(found), sw) == 0ull) {
                  if (tail_r < Q) {
                    if (is_leader) q[tail_r] = u;
                    ++tail_r;
                    wave_sync();
                    if (MODE == kModeCover && in_seed(a.seed_bits, u)) lhit = true;
                  } else {
                    lbad = true;
                  }
                }
              }
            }
          }
        }
        done_items += (uint32_t)(R * S);
      }
      wave_sync();
      const uint64_t hm = __ballot(lhit), bm = __ballot(lbad);
      hit = hit || seg_bits<S>(hm, sw) != 0ull;
      bad = bad || seg_bits<S>(bm, sw) != 0ull;
    }
  }
  flush_acc(a, blk, acc, io.acc, lane);
}

// Single launches only (launch_ic): their tiers 0 and 1 take sets from kCtrParts cursors.
// The modes that store no nodes ask for 7 wavefronts per SIMD: the 8-lane shape then fits
// 71 VGPRs without spilling and its width launches run about 3% faster.  The storing mode
// needs 80 and stays at 6 (held to 72 it spills).  Shapes with larger queues are held to 5
// or 6 by their LDS and ignore the request.
template <int MODE, bool WC, int S, int Q, int HLOG, int GMAX, int R>
__global__ __launch_bounds__(kSegThreads) __attribute__((amdgpu_waves_per_eu(MODE == kModeEmit ? 1 : 7, 8)))
void ic_seg_kernel(SampleArgs a, TierIO io) {
  __shared__ BlockAcc blk;
  block_acc_init(blk);
  ic_seg_run<MODE, WC, S, Q, HLOG, GMAX, R, true>(a, io, true, &blk);
}

// Exact sum of kappa(R) * 2^53 over the widths a width-mode launch wrote
// (Equation (8)); optionally copies the widths out as uint64.
// The block's exact sum goes to the counters with one pair of atomics (the
// wavefronts' sums meet in LDS first): atomics on one address from every
// wavefront of a large launch would serialize.
__device__ __forceinline__ void kappa_pass(const SampleArgs& a) {
  __shared__ unsigned long long s_part[kSegThreads / kWave][3];
  u128 kap = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.count; i += stride) {
    const uint32_t w = a.wbuf[i];
    kap += kappa_fixed(w, a.g.m, a.k);
    if (a.widths) a.widths[i] = w;
  }
  // 32-bit limbs and the high word summed as 64-bit values: exact for 256 lanes
  const unsigned long long lo = (unsigned long long)kap, hi = (unsigned long long)(kap >> 64);
  const unsigned long long s_hi = seg_sum<kWave>(hi);
  const unsigned long long s_l0 = seg_sum<kWave>(lo & 0xFFFFFFFFull);
  const unsigned long long s_l1 = seg_sum<kWave>(lo >> 32);
  const int wv = threadIdx.x / kWave;
  if (threadIdx.x % kWave == 0) {
    s_part[wv][0] = s_hi;
    s_part[wv][1] = s_l1;
    s_part[wv][2] = s_l0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long h = 0, l1 = 0, l0 = 0;
    for (int w = 0; w < kSegThreads / kWave; ++w) {
      h += s_part[w][0];
      l1 += s_part[w][1];
      l0 += s_part[w][2];
    }
    const u128 v = ((u128)h << 64) + ((u128)l1 << 32) + (u128)l0;
    if (v) add_u128(a.ctr + kCtrAcc + kAccKappaLo, v);
  }
}

__global__ __launch_bounds__(kSegThreads) void kappa_reduce_kernel(SampleArgs a) { kappa_pass(a); }

// ------------------------------------------------------------------------
// LT, tier 0: one chain per lane.
// ------------------------------------------------------------------------

template <int MODE>
__device__ __forceinline__ void lt_lane_run(const SampleArgs& a, const TierIO& io, BlockAcc* blk = nullptr) {
  __shared__ int32_t s_chain[kLtWaves][kChain][kWave];
  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  int32_t(*chain)[kWave] = s_chain[wv];
  const GraphView g = a.g;
  const Key key = make_key(a.seed);
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  Acc acc;
  Reservoir res;
  res.chunk = chunk_for(a.count, kLtWaves, kWave);
  if (io.parts > 1) res.part = (int)(blockIdx.x % (unsigned)kCtrParts);
  unsigned long long pool_next = 0, pool_end = 0;

  bool active = false, exhausted = false, hit = false;
  unsigned long long rel = 0, width = 0;
  int32_t v = 0;
  int len = 0;
  Sig256 sig;
  SetStream st = make_set_stream(a.phase, a.first);
  for (;;) {
    {
      unsigned long long item = 0;
      if (take(a, io.next_ctr, io.parts, a.count, res, !active && !exhausted, true, below, lane, exhausted, item)) {
        rel = item;
        st = make_set_stream(a.phase, a.first + rel);
        v = draw_root(key, st, g.n);
        chain[0][lane] = v;
        len = 1;
        width = 0;
        sig = Sig256();
        sig.add(v);
        hit = (MODE == kModeCover) && in_seed(a.seed_bits, v);
        active = true;
      }
    }
    if (__ballot(active) == 0) break;
    bool done = false, bad = false;
    if (active) {
      done = hit;
      if (!done) {
        const int64_t ea = g.off[v];
        const int64_t d = g.off[v + 1] - ea;
        width += (unsigned long long)d;
        const int64_t e = d ? lt_pick_edge(g, key, st, v, ea, d) : -1;
        if (e < 0) {
          done = true;
        } else {
          const int32_t u = g.src[e];
          bool seen = false;
          if (sig.maybe(u)) {
            for (int i = 0; i < len; ++i) {
              if (chain[i][lane] == u) {
                seen = true;
                break;
              }
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
            sig.add(u);
            v = u;
            if (MODE == kModeCover && in_seed(a.seed_bits, u)) {
              hit = true;
              done = true;
            }
          }
        }
      }
    }
    const bool fin = done && !bad;
    {
      const uint64_t dm = __ballot(bad);
      if (dm) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&a.ctr[io.out_len_ctr], (unsigned long long)__popcll(dm));
        base = lane0_u64(base);
        if (bad) {
          const unsigned long long pos = base + (unsigned long long)__popcll(dm & below);
          if (pos < a.count) io.out_list[pos] = rel;
        }
      }
    }
    if (MODE == kModeEmit) {
      const uint32_t mine = fin ? (uint32_t)len : 0u;
      const uint32_t winc = seg_incl_scan<kWave>(mine, lane);
      const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)winc, kWave - 1);
      if (tot) {
        const unsigned long long base =
            pool_place(a, (unsigned long long)a.pool_chunk, mine, winc, tot, pool_next, pool_end, lane);
        if (fin) {
          if (base + (unsigned long long)len <= a.pool_cap)
            for (int i = 0; i < len; ++i) a.pool[base + i] = chain[i][lane];
          a.set_start[rel] = a.pool_base + base;
          a.set_len[rel] = (uint32_t)len;
          if (a.widths) a.widths[rel] = width;
          if (a.wbuf) a.wbuf[rel] = (uint32_t)width;
          acc.width += width;
          acc.nodes += (unsigned long long)len;
        }
      }
    }
    if (done) {
      active = false;
      if (fin && MODE == kModeWidth) {
        a.wbuf[rel] = (uint32_t)width;
        acc.width += width;
        acc.nodes += (unsigned long long)len;
        if (a.sizes) a.sizes[rel] = (uint32_t)len;
      } else if (fin && MODE == kModeCover) {
        acc.width += width;
        acc.nodes += (unsigned long long)len;
        if (hit) acc.covered += 1;
      }
    }
  }
  flush_acc(a, blk, acc, io.acc, lane);
}

// (Per-wavefront flushes: the chains fill exactly 32 KB of LDS per block, and
// any more would cost a block per CU.)
template <int MODE>
__global__ __launch_bounds__(kLtWaves* kWave) void lt_lane_kernel(SampleArgs a, TierIO io) {
  lt_lane_run<MODE>(a, io);
}

// ------------------------------------------------------------------------
// Last tier.
// ------------------------------------------------------------------------

// IC: one 256-thread block per set, visited stamps and queue in device memory.
template <int MODE, bool WC>
__device__ __forceinline__ void ic_big_run(const SampleArgs& a, const TierIO& io, int slot) {
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
  const Key key = make_key(a.seed);
  uint32_t* stamp = a.big_stamp + (size_t)slot * (size_t)a.big_stride;
  int32_t* queue = a.big_queue + (size_t)slot * (size_t)a.big_stride;
  const unsigned long long ndef = list_len(a, io.in_len_ctr);
  Acc acc;

  for (;;) {
    if (tid == 0) {
      s_idx = atomicAdd(&a.ctr[io.next_ctr], 1ull);
      s_epoch = a.big_epoch[slot] + 1u;
    }
    __syncthreads();
    const unsigned long long idx = s_idx;
    if (idx >= ndef) break;
    uint32_t epoch = s_epoch;
    if (epoch == 0u) {  // stamp counter wrapped: start the slot afresh
      for (uint64_t i = tid; i < a.big_stride; i += T) stamp[i] = 0u;
      epoch = 1u;
    }
    const unsigned long long rel = io.in_list[idx];
    const SetStream st = make_set_stream(a.phase, a.first + rel);
    const int32_t root = draw_root(key, st, g.n);
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
      uint32_t incl = seg_incl_scan<kWave>(ng, lane);
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
          const uint4 x = draw(key, st, kKindCoin, (uint64_t)grp);
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
    const unsigned long long wsum_w = seg_sum<kWave>(wloc);
    if (lane == 0) s_red[wv] = wsum_w;
    __syncthreads();
    const uint32_t len = s_tail;
    if (MODE == kModeEmit) {
      if (tid == 0) {
        unsigned long long width = 0;
        for (int w = 0; w < T / kWave; ++w) width += s_red[w];
        const unsigned long long b = atomicAdd(&a.ctr[kCtrPoolCursor], (unsigned long long)len);
        s_base = b;
        a.set_start[rel] = a.pool_base + b;
        a.set_len[rel] = len;
        if (a.widths) a.widths[rel] = width;
        if (a.wbuf) a.wbuf[rel] = (uint32_t)width;
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
        a.wbuf[rel] = (uint32_t)width;
        acc.width += width;
        acc.nodes += len;
        if (a.sizes) a.sizes[rel] = len;
      } else {
        acc.width += width;
        acc.nodes += len;
        if (s_hit) acc.covered += 1;
      }
    }
    __syncthreads();
  }
  if (tid == 0) block_flush(a, acc, io.acc);
}

template <int MODE, bool WC>
__global__ __launch_bounds__(kBigThreads) void ic_big_kernel(SampleArgs a, TierIO io) {
  ic_big_run<MODE, WC>(a, io, blockIdx.x);
}

// ------------------------------------------------------------------------
// General triggering model (Section 4.2): every dequeued node v draws its
// triggering set T(v) from an explicit distribution over subsets of its
// in-edges (trig_pick), and the unvisited members of T(v) join the set.
// Tier 0: 16 lanes per set, four sets per wavefront, each lane taking one
// queued node of its set per step; per set a queue of 128 nodes (also the
// stored set) and an open-addressing visited hash of 256 slots in LDS.
// Tier 1: one set per wavefront, its lanes taking up to 64 queued nodes at a
// time, with a queue of 1024 and a hash of 2048.  Sets that outgrow a tier are
// deferred to the next; the last is one 512-thread block per set with visited
// stamps and a queue in device memory.
// ------------------------------------------------------------------------
constexpr int kTrigSegLanes = 16;  // lanes per set in tier 0
constexpr int kTrigSegQ = 128;     // largest set tier 0 keeps
constexpr int kTrigSegHlog = 8;    // 256 hash slots per set in tier 0
constexpr int kTrigWaves = 4;      // wavefronts per tier-1 block
constexpr int kTrigQ = 1024;       // largest set tier 1 keeps
constexpr int kTrigHlog = 11;      // 2048 hash slots per set in tier 1

template <int MODE>
__device__ __forceinline__ void trig_wave_run(const SampleArgs& a, const TierIO& io, BlockAcc* blk) {
  constexpr int H = 1 << kTrigHlog;
  __shared__ int32_t s_q[kTrigWaves][kTrigQ];
  __shared__ uint32_t s_h[kTrigWaves][H];
  __shared__ uint32_t s_tail[kTrigWaves];
  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  int32_t* q = s_q[wv];
  uint32_t* h = s_h[wv];
  const GraphView g = a.g;
  const Key key = make_key(a.seed);
  const unsigned long long total = io.in_list ? list_len(a, io.in_len_ctr) : a.count;
  Acc acc;
  Reservoir res;
  res.chunk = chunk_for(total, kTrigWaves, 1);
  if (io.parts > 1) res.part = (int)(blockIdx.x % (unsigned)kCtrParts);
  unsigned long long pool_next = 0, pool_end = 0;
  bool exhausted = false;
  for (;;) {
    unsigned long long item = 0;
    if (!take(a, io.next_ctr, io.parts, total, res, !exhausted, lane == 0, 0ull, lane, exhausted, item)) break;
    const unsigned long long rel = io.in_list ? io.in_list[item] : item;
    const SetStream st = make_set_stream(a.phase, a.first + rel);
    const int32_t root = draw_root(key, st, g.n);
    for (int i = lane; i < H; i += kWave) h[i] = 0u;
    wave_sync();
    if (lane == 0) {
      q[0] = root;
      s_tail[wv] = 1u;
      lds_insert<kTrigHlog>(h, (uint32_t)root);
    }
    wave_sync();
    bool hit = (MODE == kModeCover) && in_seed(a.seed_bits, root);
    bool bad = false;
    unsigned long long wlane = 0;
    int head = 0;
    for (;;) {
      const int tail = __builtin_amdgcn_readfirstlane((int)s_tail[wv]);
      if (head >= tail || hit || bad) break;
      const int nb = min(tail - head, kWave);
      bool lbad = false, lhit = false;
      if (lane < nb) {
        const int32_t v = q[head + lane];
        const int64_t ea = g.off[v];
        wlane += (unsigned long long)(g.off[v + 1] - ea);
        const int64_t j = trig_pick(g, key, st, v);
        if (j >= 0) {
          const int64_t m1 = g.tset[j + 1];
          for (int64_t i = g.tset[j]; i < m1; ++i) {
            const int32_t u = g.src[ea + (int64_t)g.tmem[i]];
            const int r = lds_insert<kTrigHlog>(h, (uint32_t)u);
            if (r < 0) {
              lbad = true;
              break;
            }
            if (r == 1) {
              const uint32_t pos = atomicAdd(&s_tail[wv], 1u);
              if (pos < (uint32_t)kTrigQ) q[pos] = u;
              else lbad = true;
              if (MODE == kModeCover && in_seed(a.seed_bits, u)) lhit = true;
            }
          }
        }
      }
      head += nb;
      wave_sync();
      bad = __ballot(lbad) != 0ull;
      hit = hit || __ballot(lhit) != 0ull;
    }
    const unsigned long long width = seg_sum<kWave>(wlane);
    const uint32_t len = min((uint32_t)__builtin_amdgcn_readfirstlane((int)s_tail[wv]), (uint32_t)kTrigQ);
    if (bad && !(MODE == kModeCover && hit)) {
      if (lane == 0) {
        const unsigned long long pos = atomicAdd(&a.ctr[io.out_len_ctr], 1ull);
        if (pos < a.count) io.out_list[pos] = rel;
      }
    } else if (MODE == kModeEmit) {
      const uint32_t mine = lane == 0 ? len : 0u;
      // tier 0 reserves slices; the deferral tiers (few sets) exactly what they store
      const unsigned long long slice = io.acc == 0 ? (unsigned long long)a.pool_chunk : 0ull;
      const unsigned long long my_base = pool_place(a, slice, mine, len, len, pool_next, pool_end, lane);
      const unsigned long long base = lane0_u64(my_base);
      if (base + len <= a.pool_cap)
        for (uint32_t i = lane; i < len; i += kWave) a.pool[base + i] = q[i];
      if (lane == 0) {
        a.set_start[rel] = a.pool_base + base;
        a.set_len[rel] = len;
        if (a.widths) a.widths[rel] = width;
        if (a.wbuf) a.wbuf[rel] = (uint32_t)width;
        acc.width += width;
        acc.nodes += len;
      }
    } else if (lane == 0) {
      acc.width += width;
      acc.nodes += len;
      if (MODE == kModeWidth) {
        a.wbuf[rel] = (uint32_t)width;
        if (a.sizes) a.sizes[rel] = len;
      } else if (hit) {
        acc.covered += 1;
      }
    }
    wave_sync();
  }
  flush_acc(a, blk, acc, io.acc, lane);
}

// Tier 0 of the triggering model (see above).  Its LDS admits 6 blocks of 4 wavefronts per
// CU; the request for 6 wavefronts per SIMD brings the storing mode from 81 to 79 VGPRs (it
// ran 5) without spilling, and TIM+ on this model about 1% faster.
template <int MODE>
__global__ __launch_bounds__(kSegThreads) __attribute__((amdgpu_waves_per_eu(6, 8)))
void trig_seg_kernel(SampleArgs a, TierIO io) {
  constexpr int S = kTrigSegLanes, Q = kTrigSegQ, H = 1 << kTrigSegHlog;
  constexpr int NSEG = kSegThreads / S;
  __shared__ int32_t s_q[NSEG][Q];
  __shared__ __align__(16) uint32_t s_h[NSEG][H];
  __shared__ uint32_t s_tail[NSEG];
  __shared__ BlockAcc blk;
  block_acc_init(blk);
  const int lane = threadIdx.x % kWave;
  const int sl = threadIdx.x % S;   // lane within the segment
  const int seg = threadIdx.x / S;  // segment within the block
  const int sw = lane / S;          // segment within the wavefront
  const int leader = sw * S;
  const bool is_leader = sl == 0;
  const uint64_t below_leader = leader ? (~0ull >> (64 - leader)) : 0ull;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  int32_t* q = s_q[seg];
  uint32_t* h = s_h[seg];
  uint32_t* tailp = &s_tail[seg];
  const GraphView g = a.g;
  const Key key = make_key(a.seed);
  const unsigned long long total = a.count;
  Acc acc;
  Reservoir res;
  res.chunk = chunk_for(total, kSegThreads / kWave, kWave / S);
  if (io.parts > 1) res.part = (int)(blockIdx.x % (unsigned)kCtrParts);
  RootBuffer rb;
  unsigned long long pool_next = 0, pool_end = 0;
  // segment state (the same in every lane of a segment)
  bool has = false, exhausted = false, hit = false, bad = false;
  unsigned long long rel = 0;
  SetStream st = make_set_stream(a.phase, a.first);
  int head = 0;
  unsigned long long wlane = 0;  // lane: in-degrees of the nodes it took
  for (;;) {
    // ---- A: sets whose queued nodes are all done are finished (or deferred)
    bool fin = false, defer_now = false;
    uint32_t fin_len = 0;
    unsigned long long fin_width = 0;
    if (has) {
      const int tail = (int)*tailp;
      if (bad || hit || head >= tail) {
        fin_width = seg_sum<S>(wlane);
        has = false;
        fin_len = (uint32_t)min(tail, Q);
        if (bad && !(MODE == kModeCover && hit)) {
          defer_now = true;
        } else {
          fin = true;
          if (is_leader && MODE != kModeEmit) {
            acc.width += fin_width;
            acc.nodes += fin_len;
            if (MODE == kModeWidth) {
              a.wbuf[rel] = (uint32_t)fin_width;
              if (a.sizes) a.sizes[rel] = fin_len;
            } else if (hit) {
              acc.covered += 1;
            }
          }
        }
      }
    }
    {
      const bool dl = defer_now && is_leader;
      const uint64_t dm = __ballot(dl);
      if (dm) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&a.ctr[io.out_len_ctr], (unsigned long long)__popcll(dm));
        base = lane0_u64(base);
        if (dl) {
          const unsigned long long pos = base + (unsigned long long)__popcll(dm & below);
          if (pos < a.count) io.out_list[pos] = rel;
        }
      }
    }
    if (MODE == kModeEmit) {
      const uint32_t mine = (fin && is_leader) ? fin_len : 0u;
      const uint64_t fm = __ballot(mine != 0u);
      if (fm) {
        const uint32_t winc = seg_incl_scan<kWave>(mine, lane);
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)winc, kWave - 1);
        const unsigned long long my_base =
            pool_place(a, (unsigned long long)a.pool_chunk, mine, winc, tot, pool_next, pool_end, lane);
        const unsigned long long base = __shfl(my_base, leader);
        if (fin) {
          if (base + fin_len <= a.pool_cap)
            for (uint32_t i = sl; i < fin_len; i += S) a.pool[base + i] = q[i];
          if (is_leader) {
            a.set_start[rel] = a.pool_base + base;
            a.set_len[rel] = fin_len;
            if (a.widths) a.widths[rel] = fin_width;
            if (a.wbuf) a.wbuf[rel] = (uint32_t)fin_width;
            acc.width += fin_width;
            acc.nodes += fin_len;
          }
        }
      }
    }
    wave_sync();

    // ---- B: idle segments take their next set
    {
      int32_t root = 0;
      const bool want = !has && !exhausted;
      if (take_set<true>(a, io, total, res, rb, want, is_leader, below_leader, lane, exhausted, rel, root)) {
        st = make_set_stream(a.phase, a.first + rel);
        uint4* h4 = reinterpret_cast<uint4*>(h);
        for (int i = sl; i < H / 4; i += S) h4[i] = make_uint4(0u, 0u, 0u, 0u);
        wave_sync();
        if (is_leader) {
          q[0] = root;
          *tailp = 1u;
          lds_insert<kTrigSegHlog>(h, (uint32_t)root);
        }
        has = true;
        hit = (MODE == kModeCover) && in_seed(a.seed_bits, root);
        bad = false;
        head = 0;
        wlane = 0;
      }
    }
    if (__ballot(has) == 0) break;
    wave_sync();

    // ---- C: each set's next queued nodes, one per lane: T(v) by trig_pick
    bool lbad = false, lhit = false;
    if (has && !hit && !bad) {
      const int tail = (int)*tailp;
      const int nb = min(tail - head, S);
      if (sl < nb) {
        const int32_t v = q[head + sl];
        const int64_t ea = g.off[v];
        wlane += (unsigned long long)(g.off[v + 1] - ea);
        const int64_t j = trig_pick(g, key, st, v);
        if (j >= 0) {
          const int64_t m1 = g.tset[j + 1];
          for (int64_t i = g.tset[j]; i < m1; ++i) {
            const int32_t u = g.src[ea + (int64_t)g.tmem[i]];
            const int r = lds_insert<kTrigSegHlog>(h, (uint32_t)u);
            if (r < 0) {
              lbad = true;
              break;
            }
            if (r == 1) {
              const uint32_t pos = atomicAdd(tailp, 1u);
              if (pos < (uint32_t)Q) q[pos] = u;
              else lbad = true;
              if (MODE == kModeCover && in_seed(a.seed_bits, u)) lhit = true;
            }
          }
        }
      }
      head += nb;
    }
    wave_sync();
    const uint64_t hm = __ballot(lhit), bm = __ballot(lbad);
    hit = hit || seg_bits<S>(hm, sw) != 0ull;
    bad = bad || seg_bits<S>(bm, sw) != 0ull;
  }
  flush_acc(a, &blk, acc, io.acc, lane);
}

template <int MODE>
__global__ __launch_bounds__(kTrigWaves* kWave) void trig_wave_kernel(SampleArgs a, TierIO io) {
  __shared__ BlockAcc blk;
  block_acc_init(blk);
  trig_wave_run<MODE>(a, io, &blk);
}

// Last tier of the triggering model: one block per deferred set.
template <int MODE>
__global__ __launch_bounds__(kBigThreads) void trig_big_kernel(SampleArgs a, TierIO io) {
  constexpr int T = kBigThreads;
  __shared__ unsigned long long s_red[T / kWave];
  __shared__ unsigned long long s_idx, s_base;
  __shared__ uint32_t s_tail, s_epoch;
  __shared__ int s_hit;
  const int slot = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid % kWave, wv = tid / kWave;
  const GraphView g = a.g;
  const Key key = make_key(a.seed);
  uint32_t* stamp = a.big_stamp + (size_t)slot * (size_t)a.big_stride;
  int32_t* queue = a.big_queue + (size_t)slot * (size_t)a.big_stride;
  const unsigned long long ndef = list_len(a, io.in_len_ctr);
  Acc acc;
  for (;;) {
    if (tid == 0) {
      s_idx = atomicAdd(&a.ctr[io.next_ctr], 1ull);
      s_epoch = a.big_epoch[slot] + 1u;
    }
    __syncthreads();
    const unsigned long long idx = s_idx;
    if (idx >= ndef) break;
    uint32_t epoch = s_epoch;
    if (epoch == 0u) {  // stamp counter wrapped: start the slot afresh
      for (uint64_t i = tid; i < a.big_stride; i += T) stamp[i] = 0u;
      epoch = 1u;
    }
    const unsigned long long rel = io.in_list[idx];
    const SetStream st = make_set_stream(a.phase, a.first + rel);
    const int32_t root = draw_root(key, st, g.n);
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
      const int hit = s_hit;
      __syncthreads();  // every thread has read the tail before any appends
      if (head >= tail || hit) break;
      const int64_t nb = min<int64_t>(tail - head, (int64_t)T);
      if (tid < nb) {
        const int32_t v = queue[head + tid];
        const int64_t ea = g.off[v];
        wloc += (unsigned long long)(g.off[v + 1] - ea);
        const int64_t j = trig_pick(g, key, st, v);
        if (j >= 0) {
          const int64_t m1 = g.tset[j + 1];
          for (int64_t i = g.tset[j]; i < m1; ++i) {
            const int32_t u = g.src[ea + (int64_t)g.tmem[i]];
            if (atomicExch(&stamp[u], epoch) != epoch) {
              const uint32_t pos = atomicAdd(&s_tail, 1u);
              queue[pos] = u;
              if (MODE == kModeCover && in_seed(a.seed_bits, u)) s_hit = 1;
            }
          }
        }
      }
      head += nb;
      __syncthreads();
    }
    const unsigned long long wsum_w = seg_sum<kWave>(wloc);
    if (lane == 0) s_red[wv] = wsum_w;
    __syncthreads();
    const uint32_t len = s_tail;
    unsigned long long width = 0;
    for (int w = 0; w < T / kWave; ++w) width += s_red[w];
    if (MODE == kModeEmit) {
      if (tid == 0) {
        const unsigned long long b = atomicAdd(&a.ctr[kCtrPoolCursor], (unsigned long long)len);
        s_base = b;
        a.set_start[rel] = a.pool_base + b;
        a.set_len[rel] = len;
        if (a.widths) a.widths[rel] = width;
        if (a.wbuf) a.wbuf[rel] = (uint32_t)width;
        acc.width += width;
        acc.nodes += len;
      }
      __syncthreads();
      const unsigned long long b = s_base;
      if (b + len <= a.pool_cap)
        for (uint32_t i = tid; i < len; i += T) a.pool[b + i] = queue[i];
    } else if (tid == 0) {
      acc.width += width;
      acc.nodes += len;
      if (MODE == kModeWidth) {
        a.wbuf[rel] = (uint32_t)width;
        if (a.sizes) a.sizes[rel] = len;
      } else if (s_hit) {
        acc.covered += 1;
      }
    }
    __syncthreads();
  }
  if (tid == 0) block_flush(a, acc, io.acc);
}

// LT, chains longer than the first tier's LDS chain: one lane per chain and
// no visited marks at all.  The walk's pick at a node is a fixed function of
// (set, node), so the walk is x_{i+1} = f(x_i): it ends where f stops (no
// in-edges or the empty triggering set), or it enters a cycle and the first
// repeated node closes the set.
// Brent's cycle detection (R. P. Brent, "An improved Monte Carlo
// factorization algorithm", BIT 20, 1980) finds the cycle length lambda and
// the tail length mu in O(1) memory; the set is x_0 .. x_{mu+lambda-1}, walked
// once more for its widths (and, when stored, its nodes).  Coverage needs no
// second walk: the hare of the search passes every node of the set.
//
// Every lane runs a small state machine that takes one step of f per
// iteration, so lanes of one wavefront run chains of any lengths side by
// side and take a new chain as soon as theirs is done.
enum ChainPhase : int {
  kSearch = 0,   // Brent's search: hare at position pos
  kAdvance = 1,  // hare moves lambda steps from x_0
  kTortoise = 2, // tortoise and hare step together until they meet (mu)
  kHare = 3,
  kWalk = 4,     // output walk over the mu + lambda nodes
  kIdle = 5
};

// f(v) and indeg(v): the in-neighbour the walk moves to from v, or -1 where
// the walk stops (no in-edges, or the empty triggering set).
__device__ __forceinline__ int32_t lt_next(const GraphView& g, const Key& key, const SetStream& st, int32_t v,
                                           int64_t& d) {
  const int64_t ea = g.off[v];
  d = g.off[v + 1] - ea;
  if (d == 0) return -1;
  const int64_t e = lt_pick_edge(g, key, st, v, ea, d);
  return e < 0 ? -1 : g.src[e];
}

constexpr int kChainWaves = 4;  // wavefronts per block of the long-chain tier

template <int MODE>
__device__ __forceinline__ void lt_chain_run(const SampleArgs& a, const TierIO& io, bool first_only,
                                             BlockAcc* blk = nullptr) {
  const int lane = threadIdx.x % kWave;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const GraphView g = a.g;
  const Key key = make_key(a.seed);
  const unsigned long long total = list_len(a, io.in_len_ctr);
  if (first_only) {  // a chain per lane to start with: later wavefronts are not needed
    const unsigned long long wave = (unsigned long long)blockIdx.x * kChainWaves + threadIdx.x / kWave;
    if (wave * (unsigned long long)kWave >= total) {
      flush_acc(a, blk, Acc(), io.acc, lane);
      return;
    }
  }
  Acc acc;
  Reservoir res;
  res.chunk = chunk_for(total, kChainWaves, kWave);
  bool exhausted = false;
  int phase = kIdle;
  unsigned long long rel = 0, width = 0, base = 0;
  SetStream st = make_set_stream(a.phase, a.first);
  int32_t x0 = 0, cur = 0, tort = 0, hare = 0;
  uint32_t pos = 0, power = 1, lam = 0, mu = 0, cnt = 0, len = 0;
  for (;;) {
    {
      unsigned long long item = 0;
      if (take(a, io.next_ctr, 1, total, res, phase == kIdle && !exhausted, true, below, lane, exhausted, item)) {
        rel = io.in_list[item];
        st = make_set_stream(a.phase, a.first + rel);
        x0 = draw_root(key, st, g.n);
        cur = x0;
        pos = 0;
        width = 0;
        phase = kSearch;
        if (MODE == kModeCover && in_seed(a.seed_bits, x0)) {
          acc.covered += 1;
          phase = kIdle;
        }
      }
    }
    if (__ballot(phase != kIdle) == 0) break;
    if (phase == kIdle) continue;
    const int ph = phase;  // this iteration's step is f(cur) of phase ph
    int64_t d = 0;
    const int32_t nx = lt_next(g, key, st, cur, d);
    bool done = false, walk = false;
    if (ph == kSearch) {
      // cur is the hare, at position pos
      if (nx < 0) {  // x_pos has no in-edges: the set is x_0 .. x_pos
        len = pos + 1;
        if (MODE == kModeCover) done = true;
        else walk = true;
      } else {
        if (pos == 0) {
          tort = x0;
          power = 1;
          lam = 1;
        } else {
          if (power == lam) {
            tort = cur;
            power <<= 1;
            lam = 0;
          }
          ++lam;
        }
        ++pos;
        cur = nx;
        if (MODE == kModeCover && in_seed(a.seed_bits, nx)) {
          acc.covered += 1;
          done = true;
        } else if (nx == tort) {  // a cycle of length lam; the hare has passed every node of the set
          if (MODE == kModeCover) {
            done = true;
          } else {
            phase = kAdvance;
            cnt = 0;
            cur = x0;
          }
        }
      }
    } else if (ph == kAdvance) {  // hare = x_cnt
      cur = nx;
      if (++cnt == lam) {
        hare = nx;
        tort = x0;
        mu = 0;
        if (tort == hare) {
          len = lam;
          walk = true;
        } else {
          phase = kTortoise;
          cur = tort;
        }
      }
    } else if (ph == kTortoise) {
      tort = nx;
      phase = kHare;
      cur = hare;
    } else if (ph == kHare) {
      hare = nx;
      ++mu;
      if (tort == hare) {
        len = mu + lam;
        walk = true;
      } else {
        phase = kTortoise;
        cur = tort;
      }
    } else {  // kWalk: cur = x_pos, with indeg d and successor nx
      width += (unsigned long long)d;
      if (MODE == kModeEmit && base + len <= a.pool_cap) a.pool[base + pos] = cur;
      if (++pos == len) done = true;
      else cur = nx;
    }
    if (walk) {
      phase = kWalk;
      cur = x0;
      pos = 0;
      if (MODE == kModeEmit) base = atomicAdd(&a.ctr[kCtrPoolCursor], (unsigned long long)len);
    }
    if (done) {
      phase = kIdle;
      if (MODE == kModeWidth) {
        a.wbuf[rel] = (uint32_t)width;
        acc.width += width;
        acc.nodes += len;
        if (a.sizes) a.sizes[rel] = len;
      } else if (MODE == kModeEmit) {
        a.set_start[rel] = a.pool_base + base;
        a.set_len[rel] = len;
        if (a.widths) a.widths[rel] = width;
        if (a.wbuf) a.wbuf[rel] = (uint32_t)width;
        acc.width += width;
        acc.nodes += len;
      }
    }
  }
  flush_acc(a, blk, acc, io.acc, lane);
}

template <int MODE>
__global__ __launch_bounds__(kChainWaves* kWave) void lt_chain_kernel(SampleArgs a, TierIO io) {
  __shared__ BlockAcc blk;
  block_acc_init(blk);
  lt_chain_run<MODE>(a, io, true, &blk);
}

__global__ void clear_counters_kernel(unsigned long long* ctr) {
  for (int i = threadIdx.x; i < kCtrCount; i += blockDim.x) ctr[i] = 0ull;
}

// ------------------------------------------------------------------------
// Several sampling jobs in one launch: the RR sets that many TIM+ queries
// need at one point of their runs.  A job is a whole SampleArgs (its own
// graph, keys, range of set ids, counters, node pool and deferral lists); the
// jobs of a launch share its mode and model and the last-tier slots.  Every
// wavefront (IC last tier: every block) starts on a different job and, once
// that job's cursor is spent, moves on to the next job that still has sets
// for its tier: short jobs do not leave the chip idle, and the longest job
// has every wavefront at the end.
// ------------------------------------------------------------------------

// Where tier `tier` of a job reads and sends its sets (IC: tiers 0, 1, 2;
// LT: tiers 0 and 2).
template <int MODEL>
__device__ __forceinline__ TierIO tier_io(const SampleArgs& a, int tier) {
  if (tier == 0) return TierIO{nullptr, 0, kCtrNext0, a.list1, kCtrList1, 0};
  if (MODEL == 0 && tier == 1) return TierIO{a.list1, kCtrList1, kCtrNext1, a.list2, kCtrList2, 1};
  if (MODEL == 0) return TierIO{a.list2, kCtrList2, kCtrNext2, nullptr, 0, 2};
  return TierIO{a.list1, kCtrList1, kCtrNext2, nullptr, 0, 2};
}

__device__ __forceinline__ unsigned long long load_ctr(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bit j set: job j still has unclaimed sets in `tier` (lane j looks).  A
// stale counter is never larger than the true one, so a job is never skipped
// while it has work; at worst a spent job is visited once more.
template <int MODEL>
__device__ __forceinline__ uint64_t jobs_with_work(const JobTable& t, int tier, int lane) {
  bool w = false;
  if (lane < t.njobs) {
    const SampleArgs* a = t.jobs + lane;
    unsigned long long total = a->count;
    int next = kCtrNext0;
    if (tier > 0) {
      const int len_ctr = (MODEL == 0 && tier == 2) ? kCtrList2 : kCtrList1;
      const unsigned long long d = load_ctr(a->ctr + len_ctr);
      total = d < total ? d : total;
      next = tier == 1 ? kCtrNext1 : kCtrNext2;
    }
    w = load_ctr(a->ctr + next) < total;
  }
  return __ballot(w);
}

// The job a wavefront starts with.  A wavefront leaves a job only once each
// of its segments has finished its last set there, so every move costs it
// its slowest set in flight.  Where the jobs sample one graph (t.spread), a
// set costs about the same in every job: wavefronts start spread over the
// jobs in proportion to their sets in `tier`, where their work is, and most
// make one or two moves instead of walking across every job.  Jobs of
// different graphs start with equal shares of wavefronts.
template <int MODEL>
__device__ __forceinline__ int home_job(const JobTable& t, int tier, unsigned long long wave,
                                        unsigned long long waves, int lane) {
  if (!t.spread) return (int)(wave % (unsigned long long)t.njobs);
  unsigned long long c = 0;
  if (lane < t.njobs) {
    const SampleArgs* a = t.jobs + lane;
    c = a->count;
    if (tier > 0) {
      const unsigned long long d = load_ctr(a->ctr + ((MODEL == 0 && tier == 2) ? kCtrList2 : kCtrList1));
      c = d < c ? d : c;
    }
  }
  unsigned long long incl = c;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned long long y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  const unsigned long long total = __shfl(incl, kWave - 1, kWave);
  const unsigned long long pos = total * wave / waves;  // total <= 64 * 2^26, wave < 2^31
  const int j = __popcll(__ballot(lane < t.njobs && incl <= pos));
  return j < t.njobs ? j : t.njobs - 1;
}

// The first job of mask m at or after `from`, cyclically; -1 if none.
__device__ __forceinline__ int next_job(uint64_t m, int from) {
  if (!m) return -1;
  const uint64_t hi = from < 64 ? m & (~0ull << from) : 0ull;
  return __ffsll((unsigned long long)(hi ? hi : m)) - 1;
}

template <int MODE, bool WC, int S, int Q, int HLOG, int GMAX, int R>
__global__ __launch_bounds__(kSegThreads) void ic_seg_batch_kernel(JobTable t, int tier) {
  const int lane = threadIdx.x % kWave;
  const int wave = blockIdx.x * (kSegThreads / kWave) + threadIdx.x / kWave;
  int from = home_job<0>(t, tier, (unsigned long long)wave, (unsigned long long)gridDim.x * (kSegThreads / kWave), lane);
  for (;;) {
    const int j = __builtin_amdgcn_readfirstlane(next_job(jobs_with_work<0>(t, tier, lane), from));
    if (j < 0) break;
    const SampleArgs& a = t.jobs[j];
    ic_seg_run<MODE, WC, S, Q, HLOG, GMAX, R>(a, tier_io<0>(a, tier), false);
    from = j + 1;
  }
}

template <int MODE, bool WC>
__global__ __launch_bounds__(kBigThreads) void ic_big_batch_kernel(JobTable t) {
  __shared__ int s_job;
  int from = blockIdx.x % t.njobs;
  for (;;) {
    if (threadIdx.x < kWave) {
      const int j = next_job(jobs_with_work<0>(t, 2, threadIdx.x), from);
      if (threadIdx.x == 0) s_job = j;
    }
    __syncthreads();
    const int j = __builtin_amdgcn_readfirstlane(s_job);
    __syncthreads();
    if (j < 0) break;
    const SampleArgs& a = t.jobs[j];
    ic_big_run<MODE, WC>(a, tier_io<0>(a, 2), blockIdx.x);
    from = j + 1;
  }
}

template <int MODE>
__global__ __launch_bounds__(kLtWaves* kWave) void lt_lane_batch_kernel(JobTable t) {
  const int lane = threadIdx.x % kWave;
  const int wave = blockIdx.x * kLtWaves + threadIdx.x / kWave;
  int from = home_job<1>(t, 0, (unsigned long long)wave, (unsigned long long)gridDim.x * kLtWaves, lane);
  for (;;) {
    const int j = __builtin_amdgcn_readfirstlane(next_job(jobs_with_work<1>(t, 0, lane), from));
    if (j < 0) break;
    const SampleArgs& a = t.jobs[j];
    lt_lane_run<MODE>(a, tier_io<1>(a, 0));
    from = j + 1;
  }
}

template <int MODE>
__global__ __launch_bounds__(kChainWaves* kWave) void lt_chain_batch_kernel(JobTable t) {
  const int lane = threadIdx.x % kWave;
  const int wave = blockIdx.x * kChainWaves + threadIdx.x / kWave;
  int from = home_job<1>(t, 2, (unsigned long long)wave, (unsigned long long)gridDim.x * kChainWaves, lane);
  for (;;) {
    const int j = __builtin_amdgcn_readfirstlane(next_job(jobs_with_work<1>(t, 2, lane), from));
    if (j < 0) break;
    const SampleArgs& a = t.jobs[j];
    lt_chain_run<MODE>(a, tier_io<1>(a, 2), false);
    from = j + 1;
  }
}

// kappa sums of the jobs (blockIdx.y = job); emit launches only for jobs
// that asked for them (wbuf set).
__global__ __launch_bounds__(kSegThreads) void kappa_reduce_batch_kernel(JobTable t, int emit) {
  const SampleArgs& a = t.jobs[blockIdx.y];
  if (emit && !a.wbuf) return;  // the whole block: the job stores no widths
  kappa_pass(a);
}

__global__ void clear_counters_batch_kernel(JobTable t) {
  unsigned long long* ctr = t.jobs[blockIdx.x].ctr;
  for (int i = threadIdx.x; i < kCtrCount; i += blockDim.x) ctr[i] = 0ull;
}

// ---- device-driven KptEstimation (Algorithm 2) for a batch ----
// One thread hands out this step's chunks: every query still estimating gets
// the next sets of its current round, up to job_cap, while the step's
// step_cap sets last; queries with nothing this step get an empty job.
__global__ void kpt_jobs_kernel(KptStepArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t used = 0;
  for (int j = 0; j < a.nq; ++j) {
    const KptQuery& q = a.q[j];
    SampleArgs s = SampleArgs();
    s.g = q.g;
    s.seed = q.seed;
    s.k = q.k;
    s.ctr = a.ctr + (size_t)j * kCtrCount;
    s.big_stamp = a.big_stamp;
    s.big_queue = a.big_queue;
    s.big_epoch = a.big_epoch;
    s.big_slots = a.big_slots;
    s.big_stride = a.big_stride;
    s.wbuf = a.wbuf + used;
    s.list1 = a.list1 + used;
    s.list2 = a.list2 ? a.list2 + used : nullptr;
    if (q.round > 0 && !q.err) {
      const uint64_t left = q.c[q.round] - q.pos;
      uint64_t take = left < a.job_cap ? left : a.job_cap;
      take = take < a.step_cap - used ? take : a.step_cap - used;
      s.phase = (uint32_t)q.round;
      s.first = q.pos;
      s.count = take;
      used += take;
    }
    a.jobs[j] = s;
  }
}

// One thread per query: adds the step's totals of its chunk to its round,
// and a round whose sets are all done takes the stop test of Algorithm 2.
__global__ void kpt_advance_kernel(KptStepArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.nq) return;
  KptQuery& q = a.q[j];
  const SampleArgs& s = a.jobs[j];
  if (q.round > 0 && s.count > 0) {
    const unsigned long long* h = s.ctr;
    if (h[kCtrList1] > s.count || h[kCtrList2] > s.count) q.err = 1;
    u128 sum = ((u128)q.sum_hi << 64) | (u128)q.sum_lo;
    for (int tier = 0; tier < 3; ++tier) {
      const unsigned long long* acc = h + kCtrAcc + kAccStride * tier;
      sum += ((u128)acc[kAccKappaHi] << 64) | (u128)acc[kAccKappaLo];
      q.width += acc[kAccWidth];
      q.nodes += acc[kAccNodes];
    }
    q.sum_lo = (unsigned long long)sum;
    q.sum_hi = (unsigned long long)(sum >> 64);
    q.pos += s.count;
    const int i = q.round;
    if (q.pos == q.c[i]) {
      q.r_lo[i] = q.sum_lo;
      q.r_hi[i] = q.sum_hi;
      q.r_width[i] = q.width;
      q.r_nodes[i] = q.nodes;
      // sum / c_i > 2^-i with sum = S * 2^-53: S * 2^i > c_i * 2^53 (exact)
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
  if (q.round > 0 && !q.err) atomicAdd(a.active, 1u);
}

__global__ void kpt_clear_active_kernel(unsigned int* active) {
  if (threadIdx.x == 0) *active = 0u;
}

template <typename K>
int blocks_per_cu(K kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

// Tier-0 shapes: S lanes per set, a queue of Q nodes per set in LDS (with a
// hash of 2^HLOG slots for S >= 16), and at most GMAX 4-edge groups per set
// so that wide sets, which hold a hub's long in-list, move on to a tier with
// more lanes per set instead of forming a long tail.  The hash-free shapes
// keep 16 KB of LDS per block, so a CU holds 32 wavefronts.
template <int MODE, bool WC, int S>
struct SegKernel;
template <int MODE, bool WC>
struct SegKernel<MODE, WC, 4> {
  static constexpr auto fn = ic_seg_kernel<MODE, WC, 4, 64, 0, 256, kSegGroups>;
};
template <int MODE, bool WC>
struct SegKernel<MODE, WC, 8> {
  static constexpr auto fn = ic_seg_kernel<MODE, WC, 8, 128, 0, 512, kSegGroups>;
};
template <int MODE, bool WC>
struct SegKernel<MODE, WC, 16> {
  static constexpr auto fn = ic_seg_kernel<MODE, WC, 16, 128, 8, 512, kSegGroups>;
};
template <int MODE, bool WC>
struct SegKernel<MODE, WC, 32> {
  static constexpr auto fn = ic_seg_kernel<MODE, WC, 32, 256, 9, 1024, kSegGroups>;
};
template <int MODE, bool WC>
struct SegKernel<MODE, WC, 64> {
  static constexpr auto fn = ic_seg_kernel<MODE, WC, 64, 512, 10, 2048, kSegGroups>;
};
// tier 1: one set per wavefront
template <int MODE, bool WC>
struct Tier1Kernel {
  static constexpr auto fn = ic_seg_kernel<MODE, WC, 64, 512, 10, 64 * 64, kSegGroups>;
};

void launch_kappa_reduce(const SampleArgs& a, hipStream_t s) {
  uint64_t blocks = (a.count + kSegThreads - 1) / kSegThreads;
  blocks = blocks < 1 ? 1 : (blocks > kKappaBlocks ? kKappaBlocks : blocks);
  hipLaunchKernelGGL(kappa_reduce_kernel, dim3((unsigned)blocks), dim3(kSegThreads), 0, s, a);
}

template <int MODE, bool WC>
void launch_ic(const SampleArgs& a, int S, int grid0, int grid1, hipStream_t s, hipEvent_t after0) {
  const dim3 blk(kSegThreads);
  const TierIO t0 = {nullptr, 0, kCtrNext0, a.list1, kCtrList1, 0, kCtrParts};
  const TierIO t1 = {a.list1, kCtrList1, kCtrNext1, a.list2, kCtrList2, 1, kCtrParts};
  const TierIO t2 = {a.list2, kCtrList2, kCtrNext2, nullptr, 0, 2, 1};
  switch (S) {
    case 4: hipLaunchKernelGGL((SegKernel<MODE, WC, 4>::fn), dim3(grid0), blk, 0, s, a, t0); break;
    case 8: hipLaunchKernelGGL((SegKernel<MODE, WC, 8>::fn), dim3(grid0), blk, 0, s, a, t0); break;
    case 16: hipLaunchKernelGGL((SegKernel<MODE, WC, 16>::fn), dim3(grid0), blk, 0, s, a, t0); break;
    case 32: hipLaunchKernelGGL((SegKernel<MODE, WC, 32>::fn), dim3(grid0), blk, 0, s, a, t0); break;
    default: hipLaunchKernelGGL((SegKernel<MODE, WC, 64>::fn), dim3(grid0), blk, 0, s, a, t0); break;
  }
  if (after0) (void)hipEventRecord(after0, s);
  hipLaunchKernelGGL((Tier1Kernel<MODE, WC>::fn), dim3(grid1), blk, 0, s, a, t1);
  hipLaunchKernelGGL((ic_big_kernel<MODE, WC>), dim3(a.big_slots), dim3(kBigThreads), 0, s, a, t2);
  if (MODE == kModeWidth || (MODE == kModeEmit && a.wbuf)) launch_kappa_reduce(a, s);
}

template <int MODE>
void launch_trig(const SampleArgs& a, int grid0, int grid1, hipStream_t s, hipEvent_t after0) {
  const TierIO t0 = {nullptr, 0, kCtrNext0, a.list1, kCtrList1, 0, kCtrParts};
  const TierIO t1 = {a.list1, kCtrList1, kCtrNext1, a.list2, kCtrList2, 1, kCtrParts};
  const TierIO t2 = {a.list2, kCtrList2, kCtrNext2, nullptr, 0, 2, 1};
  hipLaunchKernelGGL((trig_seg_kernel<MODE>), dim3(grid0), dim3(kSegThreads), 0, s, a, t0);
  if (after0) (void)hipEventRecord(after0, s);
  hipLaunchKernelGGL((trig_wave_kernel<MODE>), dim3(grid1), dim3(kTrigWaves * kWave), 0, s, a, t1);
  hipLaunchKernelGGL((trig_big_kernel<MODE>), dim3(a.big_slots), dim3(kBigThreads), 0, s, a, t2);
  if (MODE == kModeWidth || (MODE == kModeEmit && a.wbuf)) launch_kappa_reduce(a, s);
}

template <int MODE>
void launch_lt(const SampleArgs& a, int grid0, int grid2, hipStream_t s, hipEvent_t after0) {
  const TierIO t0 = {nullptr, 0, kCtrNext0, a.list1, kCtrList1, 0, kCtrParts};
  const TierIO t2 = {a.list1, kCtrList1, kCtrNext2, nullptr, 0, 2, 1};
  hipLaunchKernelGGL((lt_lane_kernel<MODE>), dim3(grid0), dim3(kLtWaves * kWave), 0, s, a, t0);
  if (after0) (void)hipEventRecord(after0, s);
  hipLaunchKernelGGL((lt_chain_kernel<MODE>), dim3(grid2), dim3(kChainWaves * kWave), 0, s, a, t2);
  if (MODE == kModeWidth || (MODE == kModeEmit && a.wbuf)) launch_kappa_reduce(a, s);
}

// Batched launches: 8 lanes per set in tier 0, as SegKernel<., ., 8>.
template <int MODE, bool WC>
struct BatchKernels {
  static constexpr auto seg0 = ic_seg_batch_kernel<MODE, WC, 8, 128, 0, 512, kSegGroups>;
  static constexpr auto seg1 = ic_seg_batch_kernel<MODE, WC, 64, 512, 10, 64 * 64, kSegGroups>;
};

template <int MODE, bool WC>
void launch_ic_batch(const JobTable& t, int grid0, int grid1, int slots, unsigned kappa_blocks, hipStream_t s,
                     hipEvent_t after0) {
  const dim3 blk(kSegThreads);
  hipLaunchKernelGGL((BatchKernels<MODE, WC>::seg0), dim3(grid0), blk, 0, s, t, 0);
  if (after0) (void)hipEventRecord(after0, s);
  hipLaunchKernelGGL((BatchKernels<MODE, WC>::seg1), dim3(grid1), blk, 0, s, t, 1);
  hipLaunchKernelGGL((ic_big_batch_kernel<MODE, WC>), dim3(slots), dim3(kBigThreads), 0, s, t);
  if (MODE == kModeWidth || MODE == kModeEmit)
    hipLaunchKernelGGL(kappa_reduce_batch_kernel, dim3(kappa_blocks, t.njobs), blk, 0, s, t, MODE == kModeEmit ? 1 : 0);
}

template <int MODE>
void launch_lt_batch(const JobTable& t, int grid0, int grid2, unsigned kappa_blocks, hipStream_t s, hipEvent_t after0) {
  hipLaunchKernelGGL((lt_lane_batch_kernel<MODE>), dim3(grid0), dim3(kLtWaves * kWave), 0, s, t);
  if (after0) (void)hipEventRecord(after0, s);
  hipLaunchKernelGGL((lt_chain_batch_kernel<MODE>), dim3(grid2), dim3(kChainWaves * kWave), 0, s, t);
  if (MODE == kModeWidth || MODE == kModeEmit)
    hipLaunchKernelGGL(kappa_reduce_batch_kernel, dim3(kappa_blocks, t.njobs), dim3(kSegThreads), 0, s, t,
                       MODE == kModeEmit ? 1 : 0);
}

template <int MODE, bool WC>
int ic_occupancy(int S) {
  switch (S) {
    case 4: return blocks_per_cu((SegKernel<MODE, WC, 4>::fn), kSegThreads);
    case 8: return blocks_per_cu((SegKernel<MODE, WC, 8>::fn), kSegThreads);
    case 16: return blocks_per_cu((SegKernel<MODE, WC, 16>::fn), kSegThreads);
    case 32: return blocks_per_cu((SegKernel<MODE, WC, 32>::fn), kSegThreads);
    default: return blocks_per_cu((SegKernel<MODE, WC, 64>::fn), kSegThreads);
  }
}

}  // namespace

void launch_clear_counters(unsigned long long* ctr, hipStream_t s) {
  hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(64), 0, s, ctr);
}

int ic_seg_lanes() {
  const char* e = getenv("TIM_IC_SEG_LANES");
  const int v = e ? atoi(e) : 8;
  return (v == 4 || v == 8 || v == 16 || v == 32 || v == 64) ? v : 8;
}

int ic_tier1_blocks_per_cu(int mode, bool wc) {
  switch (mode * 2 + (wc ? 1 : 0)) {
    case 0: return blocks_per_cu((Tier1Kernel<kModeWidth, false>::fn), kSegThreads);
    case 1: return blocks_per_cu((Tier1Kernel<kModeWidth, true>::fn), kSegThreads);
    case 2: return blocks_per_cu((Tier1Kernel<kModeEmit, false>::fn), kSegThreads);
    case 3: return blocks_per_cu((Tier1Kernel<kModeEmit, true>::fn), kSegThreads);
    case 4: return blocks_per_cu((Tier1Kernel<kModeCover, false>::fn), kSegThreads);
    default: return blocks_per_cu((Tier1Kernel<kModeCover, true>::fn), kSegThreads);
  }
}

int ic_blocks_per_cu(int mode, bool wc, int S) {
  switch (mode * 2 + (wc ? 1 : 0)) {
    case 0: return ic_occupancy<kModeWidth, false>(S);
    case 1: return ic_occupancy<kModeWidth, true>(S);
    case 2: return ic_occupancy<kModeEmit, false>(S);
    case 3: return ic_occupancy<kModeEmit, true>(S);
    case 4: return ic_occupancy<kModeCover, false>(S);
    default: return ic_occupancy<kModeCover, true>(S);
  }
}

int lt_chain_blocks_per_cu(int mode, bool batch) {
  switch (mode + (batch ? 3 : 0)) {
    case 0: return blocks_per_cu(lt_chain_kernel<kModeWidth>, kChainWaves * kWave);
    case 1: return blocks_per_cu(lt_chain_kernel<kModeEmit>, kChainWaves * kWave);
    case 2: return blocks_per_cu(lt_chain_kernel<kModeCover>, kChainWaves * kWave);
    case 3: return blocks_per_cu(lt_chain_batch_kernel<kModeWidth>, kChainWaves * kWave);
    case 4: return blocks_per_cu(lt_chain_batch_kernel<kModeEmit>, kChainWaves * kWave);
    default: return blocks_per_cu(lt_chain_batch_kernel<kModeCover>, kChainWaves * kWave);
  }
}

int lt_lane_blocks_per_cu(int mode) {
  switch (mode) {
    case 0: return blocks_per_cu(lt_lane_kernel<kModeWidth>, kLtWaves * kWave);
    case 1: return blocks_per_cu(lt_lane_kernel<kModeEmit>, kLtWaves * kWave);
    default: return blocks_per_cu(lt_lane_kernel<kModeCover>, kLtWaves * kWave);
  }
}

int trig_blocks_per_cu(int mode) {
  switch (mode) {
    case 0: return blocks_per_cu(trig_seg_kernel<kModeWidth>, kSegThreads);
    case 1: return blocks_per_cu(trig_seg_kernel<kModeEmit>, kSegThreads);
    default: return blocks_per_cu(trig_seg_kernel<kModeCover>, kSegThreads);
  }
}

int trig_tier1_blocks_per_cu(int mode) {
  switch (mode) {
    case 0: return blocks_per_cu(trig_wave_kernel<kModeWidth>, kTrigWaves * kWave);
    case 1: return blocks_per_cu(trig_wave_kernel<kModeEmit>, kTrigWaves * kWave);
    default: return blocks_per_cu(trig_wave_kernel<kModeCover>, kTrigWaves * kWave);
  }
}

uint32_t tier0_set_cap(int model, int seg_lanes) {
  if (model == 1) return (uint32_t)kChain;
  if (model == 2) return (uint32_t)kTrigSegQ;
  switch (seg_lanes) {
    case 4: return 64;
    case 8: return 128;
    case 16: return 128;
    case 32: return 256;
    default: return 512;
  }
}

int batch_blocks_per_cu(int model, int mode, bool wc, int tier) {
  if (model == 1) {
    switch (mode) {
      case 0: return blocks_per_cu(lt_lane_batch_kernel<kModeWidth>, kLtWaves * kWave);
      case 1: return blocks_per_cu(lt_lane_batch_kernel<kModeEmit>, kLtWaves * kWave);
      default: return blocks_per_cu(lt_lane_batch_kernel<kModeCover>, kLtWaves * kWave);
    }
  }
  switch (mode * 2 + (wc ? 1 : 0) + (tier ? 6 : 0)) {
    case 0: return blocks_per_cu((BatchKernels<kModeWidth, false>::seg0), kSegThreads);
    case 1: return blocks_per_cu((BatchKernels<kModeWidth, true>::seg0), kSegThreads);
    case 2: return blocks_per_cu((BatchKernels<kModeEmit, false>::seg0), kSegThreads);
    case 3: return blocks_per_cu((BatchKernels<kModeEmit, true>::seg0), kSegThreads);
    case 4: return blocks_per_cu((BatchKernels<kModeCover, false>::seg0), kSegThreads);
    case 5: return blocks_per_cu((BatchKernels<kModeCover, true>::seg0), kSegThreads);
    case 6: return blocks_per_cu((BatchKernels<kModeWidth, false>::seg1), kSegThreads);
    case 7: return blocks_per_cu((BatchKernels<kModeWidth, true>::seg1), kSegThreads);
    case 8: return blocks_per_cu((BatchKernels<kModeEmit, false>::seg1), kSegThreads);
    case 9: return blocks_per_cu((BatchKernels<kModeEmit, true>::seg1), kSegThreads);
    case 10: return blocks_per_cu((BatchKernels<kModeCover, false>::seg1), kSegThreads);
    default: return blocks_per_cu((BatchKernels<kModeCover, true>::seg1), kSegThreads);
  }
}

void launch_kpt_jobs(const KptStepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(kpt_jobs_kernel, dim3(1), dim3(64), 0, s, a);
}

void launch_kpt_advance(const KptStepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(kpt_clear_active_kernel, dim3(1), dim3(64), 0, s, a.active);
  hipLaunchKernelGGL(kpt_advance_kernel, dim3((unsigned)((a.nq + 63) / 64)), dim3(64), 0, s, a);
}

void launch_clear_counters_batch(const JobTable& t, hipStream_t s) {
  hipLaunchKernelGGL(clear_counters_batch_kernel, dim3(t.njobs), dim3(64), 0, s, t);
}

void launch_sample_batch(int model, int mode, bool wc, const JobTable& t, int grid0, int grid1, int slots,
                         uint64_t max_count, hipStream_t s, hipEvent_t after_tier0) {
  uint64_t kb = (max_count + kSegThreads - 1) / kSegThreads;
  const unsigned kappa_blocks = (unsigned)(kb < 1 ? 1 : (kb > kKappaBlocks ? kKappaBlocks : kb));
  if (model == 0) {
    switch (mode * 2 + (wc ? 1 : 0)) {
      case 0: launch_ic_batch<kModeWidth, false>(t, grid0, grid1, slots, kappa_blocks, s, after_tier0); break;
      case 1: launch_ic_batch<kModeWidth, true>(t, grid0, grid1, slots, kappa_blocks, s, after_tier0); break;
      case 2: launch_ic_batch<kModeEmit, false>(t, grid0, grid1, slots, kappa_blocks, s, after_tier0); break;
      case 3: launch_ic_batch<kModeEmit, true>(t, grid0, grid1, slots, kappa_blocks, s, after_tier0); break;
      case 4: launch_ic_batch<kModeCover, false>(t, grid0, grid1, slots, kappa_blocks, s, after_tier0); break;
      default: launch_ic_batch<kModeCover, true>(t, grid0, grid1, slots, kappa_blocks, s, after_tier0); break;
    }
  } else {
    switch (mode) {
      case 0: launch_lt_batch<kModeWidth>(t, grid0, grid1, kappa_blocks, s, after_tier0); break;
      case 1: launch_lt_batch<kModeEmit>(t, grid0, grid1, kappa_blocks, s, after_tier0); break;
      default: launch_lt_batch<kModeCover>(t, grid0, grid1, kappa_blocks, s, after_tier0); break;
    }
  }
}

void launch_sample(int model, int mode, const SampleArgs& a, int seg_lanes, int grid0, int grid1, hipStream_t s,
                   hipEvent_t after_tier0) {
  if (model == 0) {
    const int S = seg_lanes;
    const bool wc = a.g.thr == nullptr;
    switch (mode * 2 + (wc ? 1 : 0)) {
      case 0: launch_ic<kModeWidth, false>(a, S, grid0, grid1, s, after_tier0); break;
      case 1: launch_ic<kModeWidth, true>(a, S, grid0, grid1, s, after_tier0); break;
      case 2: launch_ic<kModeEmit, false>(a, S, grid0, grid1, s, after_tier0); break;
      case 3: launch_ic<kModeEmit, true>(a, S, grid0, grid1, s, after_tier0); break;
      case 4: launch_ic<kModeCover, false>(a, S, grid0, grid1, s, after_tier0); break;
      default: launch_ic<kModeCover, true>(a, S, grid0, grid1, s, after_tier0); break;
    }
  } else if (model == 2) {
    switch (mode) {
      case 0: launch_trig<kModeWidth>(a, grid0, grid1, s, after_tier0); break;
      case 1: launch_trig<kModeEmit>(a, grid0, grid1, s, after_tier0); break;
      default: launch_trig<kModeCover>(a, grid0, grid1, s, after_tier0); break;
    }
  } else {
    switch (mode) {
      case 0: launch_lt<kModeWidth>(a, grid0, grid1, s, after_tier0); break;
      case 1: launch_lt<kModeEmit>(a, grid0, grid1, s, after_tier0); break;
      default: launch_lt<kModeCover>(a, grid0, grid1, s, after_tier0); break;
    }
  }
}

}  // namespace tim
