// sdtw_argmin.hpp -- reduction of the last DP row of a query to
// (cost, end_pos).
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

// Block-wide lexicographic argmin of row[0..m); every thread gets the result.
// Written without thread-dependent branches (all lanes of a wave hold the
// same value after the butterfly and store it together), so it can sit in a
// loop that also holds barriers.
__device__ __forceinline__ ValIdx block_argmin(const float* __restrict__ row, int m) {
  __shared__ ValIdx s_part[1024 / kWave];
  ValIdx x{inf_f32(), 0x7fffffff};
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const float v = row[j];
    if (v < x.v) { x.v = v; x.i = j; }     // j increases: keeps the first minimiser
  }
  x = wave_argmin(x);
  const int nw = (int)(blockDim.x / kWave);
  s_part[threadIdx.x / kWave] = x;
  __syncthreads();
  x = s_part[0];
  for (int k = 1; k < nw; ++k) x = better(x, s_part[k]);
  __syncthreads();
  return x;
}

}  // namespace sdtw
