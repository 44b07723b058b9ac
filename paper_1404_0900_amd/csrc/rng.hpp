// Counter-based random numbers for the RR-set samplers.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications, the key bumped by the Weyl constants between
// rounds.  One block of four 32-bit words is addressed by
//   key     = (seed lo, seed hi)
//   counter = (idx lo, phase<<24 | kind<<16 | idx bits 32..47, set lo, set hi)
// so every coin, root and LT pick is a pure function of (seed, phase, set,
// what is drawn), and a set can be regenerated bit-exactly anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tim {

enum : uint32_t { kKindRoot = 0, kKindCoin = 1, kKindPick = 2, kKindTrigger = 3 };

__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
  k0 = __builtin_amdgcn_readfirstlane(k0);
  k1 = __builtin_amdgcn_readfirstlane(k1);
  asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 product per multiplier: a single v_mad_u64_u32 each
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// The key: the same for every set of a launch (kept in scalar registers).
struct Key {
  uint32_t k0, k1;
};

__device__ __forceinline__ Key make_key(uint64_t seed) {
  Key k;
  k.k0 = (uint32_t)seed;
  k.k1 = (uint32_t)(seed >> 32);
  return k;
}

// The part of a counter that is fixed for one RR set.
struct SetStream {
  uint32_t phase_bits;  // phase << 24
  uint32_t s_lo, s_hi;  // set id
};

__device__ __forceinline__ SetStream make_set_stream(uint32_t phase, uint64_t set) {
  SetStream st;
  st.phase_bits = phase << 24;
  st.s_lo = (uint32_t)set;
  st.s_hi = (uint32_t)(set >> 32);
  return st;
}

__device__ __forceinline__ uint4 draw(const Key& key, const SetStream& st, uint32_t kind, uint64_t idx) {
  const uint4 c = make_uint4((uint32_t)idx, st.phase_bits | (kind << 16) | ((uint32_t)(idx >> 32) & 0xFFFFu),
                             st.s_lo, st.s_hi);
  return philox10(c, key.k0, key.k1);
}

// floor(X64 * r / 2^64) with X64 = word1:word0 — a uniform index in [0, r).
__device__ __forceinline__ uint64_t scale64(uint4 x, uint64_t r) {
  const uint64_t x64 = ((uint64_t)x.y << 32) | x.x;
  return __umul64hi(x64, r);
}

// Uniform root of the set (Definition 2).
__device__ __forceinline__ int32_t draw_root(const Key& key, const SetStream& st, int64_t n) {
  return (int32_t)scale64(draw(key, st, kKindRoot, 0), (uint64_t)n);
}

}  // namespace tim
