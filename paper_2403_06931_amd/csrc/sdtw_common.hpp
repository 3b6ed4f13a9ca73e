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
constexpr int kRowCkpt = 256;        // row checkpoints: D(256k, 1..M) for 256k < N
constexpr int kSquared = 0;
constexpr int kAbsolute = 1;
// Squared difference with early pruning (the paper's Section 8 proposal):
// after the subtraction, a pair farther apart than the threshold tau is
// treated as unable to lie on the path and costs +inf, with no
// multiplication; otherwise the cost is t*t.
constexpr int kPruned = 2;

__device__ __forceinline__ float inf_f32() { return __builtin_huge_valf(); }

// Local cost c(q, r) for the cost kind (tau: the pruning threshold, used by
// kPruned only).
template <int KIND>
__device__ __forceinline__ float local_cost(float q, float r, float tau = 0.0f) {
  float t = q - r;
  if constexpr (KIND == kSquared) {
    return t * t;
  } else if constexpr (KIND == kPruned) {
    // Without a compare: (|t| - tau) * inf is +inf when |t| > tau, -inf when
    // |t| < tau and NaN when they are equal (the difference of two binary32
    // values is zero only when they are equal, subnormals being kept), and
    // the IEEE maximum ignores a NaN operand.  Every instruction reads only
    // vector registers, so all of them can dual-issue; a compare and select
    // would go through VCC, which cannot.
    const float w = (__builtin_fabsf(t) - tau) * inf_f32();
    return __builtin_fmaxf(t * t, w);
  } else {
    return __builtin_fabsf(t);
  }
}

// A wave-uniform value moved into a vector register.  The compiler would
// keep it in a scalar register, and VALU instructions that read a scalar
// register are not dual-issued on gfx950.
__device__ __forceinline__ float vgpr_copy(float x) {
  float v;
  asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
  return v;
}

// Exact three-way minimum (one v_min3_f32).  Inputs are never NaN here: DP
// values start at 0 or +inf and every LDS slot a lane reads before its
// first tile is initialised (+inf boundaries, a zeroed reference ring).
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
