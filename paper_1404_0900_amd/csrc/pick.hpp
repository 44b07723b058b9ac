// The live-edge rules of the two models, shared by the RR-set samplers
// (reverse) and the spread evaluator (forward), so that both see the same
// world for the same (seed, phase, set): IC edges by their coin words and
// thresholds (Section 2.1), LT by the one in-edge each node picks (Section 4.2;
// Section 7.1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.hpp"
#include "rng.hpp"

namespace tim {

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

// The in-edge an LT walk takes at v (in-degree d >= 1, first in-edge ea), or
// -1 if it stops there.  With 1/indeg weights: in-edge floor(X64 * d / 2^64).
// With cumulative thresholds t (Section 7.1's normalized random weights): the
// first in-edge j with word0 <= t_j, found by binary search over v's list; the
// walk stops if word0 exceeds t_{d-1} (weights summing below 1).
__device__ __forceinline__ int64_t lt_pick_edge(const GraphView& g, const Key& key, const SetStream& st, int32_t v,
                                                int64_t ea, int64_t d) {
  const uint4 x = draw(key, st, kKindPick, (uint64_t)v);
  if (!g.lthr) return ea + (int64_t)scale64(x, (uint64_t)d);
  const uint32_t* t = g.lthr + ea;
  if (x.x > t[d - 1]) return -1;
  int64_t lo = 0, hi = d - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (x.x <= t[mid]) hi = mid;
    else lo = mid + 1;
  }
  return ea + lo;
}

// General triggering model (Section 4.2): the outcome node v draws from its
// explicit distribution (an index into g.tthr / g.tset), or -1 for the empty
// triggering set.  The outcomes of v are [toff[v], toff[v+1]) with
// non-decreasing cumulative thresholds; with x = word 0 of v's draw of kind
// 3, the first outcome with x <= its threshold, found by binary search.
__device__ __forceinline__ int64_t trig_pick(const GraphView& g, const Key& key, const SetStream& st, int32_t v) {
  int64_t lo = g.toff[v];
  const int64_t end = g.toff[v + 1];
  if (lo == end) return -1;
  const uint32_t x = draw(key, st, kKindTrigger, (uint64_t)v).x;
  if (x > g.tthr[end - 1]) return -1;
  int64_t hi = end - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (x <= g.tthr[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

}  // namespace tim
