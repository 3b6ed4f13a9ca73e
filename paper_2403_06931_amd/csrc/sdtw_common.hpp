// sdtw_common.hpp -- device-side building blocks shared by the sDTW kernels.
//
// The DP cell (paper: Section 2, Eq. (1)):
//     D(i,j) = min{D(i-1,j), D(i,j-1), D(i-1,j-1)} + c(q_i, r_j)
// evaluated in binary32 as t = q - r; c = t*t (or |t|); D = min3 + c, every
// operation rounded to nearest-even (the library is built with
// -ffp-contract=off so no fused multiply-add is formed).  Each cell is a
// deterministic function of its three inputs, so any schedule of the cells
// yields identical bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdtw {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kSquared = 0;
constexpr int kAbsolute = 1;

__device__ __forceinline__ float inf_f32() { return __builtin_huge_valf(); }

// Local cost c(q, r) for the cost kind.
template <int KIND>
__device__ __forceinline__ float local_cost(float q, float r) {
  float t = q - r;
  if constexpr (KIND == kSquared) {
    return t * t;
  } else {
    return __builtin_fabsf(t);
  }
}

// Exact three-way minimum (one v_min3_f32).  Inputs are never NaN here.
__device__ __forceinline__ float min3(float a, float b, float c) {
  return __builtin_fminf(__builtin_fminf(a, b), c);
}

// Wavefront right shift by one lane (DPP wave_shr:1): lane l receives lane
// l-1's `v`; lane 0 keeps `lane0` (the row mask and bank mask enable every
// lane, and bound_ctrl is off so the invalid source lane leaves the old
// value in place).
__device__ __forceinline__ float wave_shr1(float lane0, float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, lane0),
                                         __builtin_bit_cast(int, v),
                                         0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}

template <int X>
constexpr int pow2_ceil() {
  int p = 1;
  while (p < X) p <<= 1;
  return p;
}

}  // namespace sdtw
