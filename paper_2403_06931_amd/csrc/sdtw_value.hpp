// sdtw_value.hpp -- the value a DP lane row carries, and its cell arithmetic.
//
//   float   one query per lane row, binary32 (the library's default path);
//   f16x2   two queries per lane row, one per 16-bit half, in binary16: the
//           paper's own precision and packing (Section 5.2 converts the
//           inputs to half precision and works on pairs of them; Section 8
//           names the half2 arithmetic as the kernel's main speed lever).
//           Here the two halves hold the same row of two different queries
//           of equal length, so both halves see the same reference value
//           and the same neighbours: every packed operation does two cells
//           of unrelated DPs, with no shuffling between halves.
//   Code8   one query per lane row, on uint8 codes (Section 8's proposed
//           quantisation), the DP in binary32 with the local cost (a - b)^2.
//
// Each packed operation rounds each half to nearest-even binary16, with
// subnormals kept; the minimum is exact.
#pragma once

#include "sdtw_common.hpp"

namespace sdtw {

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

template <typename V>
struct Val;

template <>
struct Val<float> {
  using In = float;                            // element type in HBM
  static constexpr int N = 1;                  // queries per value
  static constexpr bool kAntiDiagonal = false; // cell order in a step's block
  __device__ static float inf() { return inf_f32(); }
  __device__ static float zero() { return 0.0f; }
  __device__ static float query(float a, float) { return a; }
  __device__ static float ref(float r) { return r; }
  template <int KIND>
  __device__ static float cost(float q, float r, float tau) { return local_cost<KIND>(q, r, tau); }
  __device__ static float min3(float a, float b, float c) { return sdtw::min3(a, b, c); }
  __device__ static float add(float a, float b) { return a + b; }
  template <int KIND>
  __device__ static float cell(float q, float r, float up, float left, float diag, float tau) {
    const float c = cost<KIND>(q, r, tau);
    return min3(up, left, diag) + c;
  }
  __device__ static float shr1(float lane0, float v) { return wave_shr1(lane0, v); }
  __device__ static float half(float v, int) { return v; }
};

template <>
struct Val<f16x2> {
  using In = float;
  static constexpr int N = 2;
  static constexpr bool kAntiDiagonal = true;
  __device__ static f16x2 inf() {
    const _Float16 h = (_Float16)__builtin_huge_valf();
    return f16x2{h, h};
  }
  __device__ static f16x2 zero() { return f16x2{(_Float16)0.0f, (_Float16)0.0f}; }
  // the two queries' values, rounded to binary16
  __device__ static f16x2 query(float a, float b) { return f16x2{(_Float16)a, (_Float16)b}; }
  // one reference value for both halves
  __device__ static f16x2 ref(float r) {
    const _Float16 h = (_Float16)r;
    return f16x2{h, h};
  }
  template <int KIND>
  __device__ static f16x2 cost(f16x2 q, f16x2 r, float) {
    static_assert(KIND != kPruned, "pruning is a binary32 cost kind");
    const f16x2 t = q - r;                     // v_pk_add_f16 with a negated operand
    if constexpr (KIND == kSquared) {
      return t * t;                            // v_pk_mul_f16
    } else {
      // |t|: clear both sign bits
      return __builtin_bit_cast(f16x2, __builtin_bit_cast(uint32_t, t) & 0x7fff7fffu);
    }
  }
  // DP values are never negative or NaN, and the bit patterns of binary16
  // values >= +0 (up to +inf) order like the values, so an unsigned 16-bit
  // minimum per half is the exact minimum (v_pk_min_u16; a floating-point
  // minimum would first have to quiet signalling NaNs, an extra instruction
  // per operand that comes from memory or a lane move).
  __device__ static f16x2 min3(f16x2 a, f16x2 b, f16x2 c) {
    const u16x2 m = __builtin_elementwise_min(
        __builtin_elementwise_min(__builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)),
        __builtin_bit_cast(u16x2, c));
    return __builtin_bit_cast(f16x2, m);
  }
  __device__ static f16x2 add(f16x2 a, f16x2 b) { return a + b; }          // v_pk_add_f16
  template <int KIND>
  __device__ static f16x2 cell(f16x2 q, f16x2 r, f16x2 up, f16x2 left, f16x2 diag, float tau) {
    const f16x2 c = cost<KIND>(q, r, tau);
    return add(min3(up, left, diag), c);
  }
  __device__ static f16x2 shr1(f16x2 lane0, f16x2 v) {
    return __builtin_bit_cast(
        f16x2, wave_shr1(__builtin_bit_cast(float, lane0), __builtin_bit_cast(float, v)));
  }
  __device__ static float half(f16x2 v, int h) { return (float)(h == 0 ? v.x : v.y); }
};

// DP on uint8 codes, in binary32.  A code difference is an integer of at
// most 255 in magnitude, so t*t <= 65025 is exact in binary32 and one fused
// multiply-add, D = fma(t, t, min3), rounds exactly like the separate
// product and sum: the cell is three binary32 instructions (v_sub_f32,
// v_min3_f32, v_fma_f32), all of which can dual-issue, and the values equal
// the binary32 DP of the codes taken as floats (exact integers while the
// sums stay below 2^24).  +inf absorbs as in the binary32 path.
struct Code8 {
  float v;
};

template <>
struct Val<Code8> {
  using In = uint8_t;
  static constexpr int N = 1;
  static constexpr bool kAntiDiagonal = false;  // measured: row order is as fast
  __device__ static Code8 inf() { return Code8{inf_f32()}; }
  __device__ static Code8 zero() { return Code8{0.0f}; }
  __device__ static Code8 query(uint8_t a, uint8_t) { return Code8{(float)a}; }
  __device__ static Code8 ref(uint8_t r) { return Code8{(float)r}; }
  template <int KIND>
  __device__ static Code8 cell(Code8 q, Code8 r, Code8 up, Code8 left, Code8 diag, float) {
    static_assert(KIND == kSquared, "codes use the squared difference");
    const float t = q.v - r.v;                   // exact
    return Code8{__builtin_fmaf(t, t, sdtw::min3(up.v, left.v, diag.v))};
  }
  __device__ static Code8 shr1(Code8 lane0, Code8 v) {
    return Code8{wave_shr1(lane0.v, v.v)};
  }
  __device__ static float half(Code8 v, int) { return v.v; }
};

}  // namespace sdtw
