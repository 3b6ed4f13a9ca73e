// sdtw_argmin.hpp -- lexicographic (value, index) reduction used to turn the
// last DP row of a query into (cost, end_pos).
//
// cost = min_j D(N,j), end_pos = smallest 0-based j attaining it (the
// walk-back of Section 2 starts from the minimum of the last row; Section 5.2
// reduces that row to its minimum).  The reduction compares (value, index)
// pairs lexicographically, so the result does not depend on the reduction
// order.
#pragma once

#include "sdtw_common.hpp"

namespace sdtw {

struct ValIdx {
  float v;
  int32_t i;
};

__device__ __forceinline__ ValIdx better(ValIdx a, ValIdx b) {
  if (b.v < a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

__device__ __forceinline__ ValIdx wave_argmin(ValIdx x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    ValIdx o;
    o.v = __shfl_xor(x.v, d, kWave);
    o.i = __shfl_xor(x.i, d, kWave);
    x = better(x, o);
  }
  return x;
}

}  // namespace sdtw
