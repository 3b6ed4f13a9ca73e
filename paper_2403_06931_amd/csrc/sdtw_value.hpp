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
//   uint32_t  one query per lane row, on uint8 codes (Section 8's proposed
//           quantisation): the local cost (a - b)^2 and the DP run exactly in
//           32-bit integers (v_sub_u32, v_mul_i32_i24, v_min3_u32, v_add_u32,
//           all full-rate and dual-issuable like their binary32 twins).
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
  static constexpr bool kZeroRing = false;     // +inf absorbs any cost
  __device__ static float inf() { return inf_f32(); }
  __device__ static float zero() { return 0.0f; }
  __device__ static float query(float a, float) { return a; }
  __device__ static float ref(float r) { return r; }
  template <int KIND>
  __device__ static float cost(float q, float r, float tau) { return local_cost<KIND>(q, r, tau); }
  __device__ static float min3(float a, float b, float c) { return sdtw::min3(a, b, c); }
  __device__ static float add(float a, float b) { return a + b; }
  __device__ static float shr1(float lane0, float v) { return wave_shr1(lane0, v); }
  __device__ static float half(float v, int) { return v; }
};

template <>
struct Val<f16x2> {
  using In = float;
  static constexpr int N = 2;
  static constexpr bool kZeroRing = false;
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
  __device__ static f16x2 shr1(f16x2 lane0, f16x2 v) {
    return __builtin_bit_cast(
        f16x2, wave_shr1(__builtin_bit_cast(float, lane0), __builtin_bit_cast(float, v)));
  }
  __device__ static float half(f16x2 v, int h) { return (float)(h == 0 ? v.x : v.y); }
};

// Integer DP on codes.  "Infinity" is 0x7f800000, the bit pattern of
// binary32 +inf: below it, non-negative 32-bit integers order like the
// binary32 values with the same bits, so the last-row fold and its result
// move through the binary32 paths unchanged.  Every computed cell of a query
// of n rows is at most n * 255^2 (the path down the diagonal or a column), so
// finite values stay below 0x7f800000 for n <= 32,768.  Cells that the
// schedule computes before a lane's first real tile start from the boundary
// value and only grow, so they never undercut a real one -- provided every
// local cost stays at most 255^2: the reference ring is zeroed before each
// pass (kZeroRing), since an unwritten slot read by such a cell would give an
// arbitrary 32-bit product and a sum that wraps.  With costs bounded, those
// cells grow by at most 255^2 per column over a fill of at most ~10^4
// columns, far from wrapping past 2^32.
template <>
struct Val<uint32_t> {
  using In = uint8_t;
  static constexpr int N = 1;
  static constexpr bool kZeroRing = true;
  __device__ static uint32_t inf() { return 0x7f800000u; }
  __device__ static uint32_t zero() { return 0u; }
  __device__ static uint32_t query(uint8_t a, uint8_t) { return a; }
  __device__ static uint32_t ref(uint8_t r) { return r; }
  template <int KIND>
  __device__ static uint32_t cost(uint32_t q, uint32_t r, float) {
    static_assert(KIND == kSquared, "codes use the squared difference");
    const int t = (int)q - (int)r;               // |t| <= 255: a 24-bit product
    return (uint32_t)__mul24(t, t);
  }
  __device__ static uint32_t min3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_elementwise_min(__builtin_elementwise_min(a, b), c);
  }
  __device__ static uint32_t add(uint32_t a, uint32_t b) { return a + b; }
  __device__ static uint32_t shr1(uint32_t lane0, uint32_t v) {
    return __builtin_bit_cast(
        uint32_t, wave_shr1(__builtin_bit_cast(float, lane0), __builtin_bit_cast(float, v)));
  }
  __device__ static float half(uint32_t v, int) { return __builtin_bit_cast(float, v); }
};

}  // namespace sdtw
