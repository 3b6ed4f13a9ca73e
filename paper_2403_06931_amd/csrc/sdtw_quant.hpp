// sdtw_quant.hpp -- uint8 codebook quantisation of queries and reference
// (Section 8's proposal: a codebook built from the distribution of the
// reference's values, its bulk divided evenly over the 256 codes, outliers
// clamped to the end codes).  Included by the API translation unit only.
//
// Codebook.  The inputs are z-normalised, so the bulk of the reference's
// distribution is taken as the values within kU8Clip standard deviations of
// its mean: lo = max(min(reference), -kU8Clip), hi = min(max(reference),
// kU8Clip), with 256 evenly spaced levels lo + k (hi - lo) / 255.  A minimum
// and a maximum do not depend on the order of the reduction, so the codebook
// is reproducible bit for bit.
//
// Codes.  code(x) = clamp(rint((x - lo) * scale), 0, 255) with
// scale = 255 / (hi - lo), in binary64 (round half to even); a degenerate
// codebook (hi <= lo) maps everything to code 0.
#pragma once

#include "sdtw_common.hpp"

namespace sdtw {

constexpr float kU8Clip = 4.0f;
constexpr int kQThreads = 256;
constexpr int kQPer = 16;                        // elements per thread, min/max pass
constexpr int kQChunk = kQThreads * kQPer;       // elements per workgroup

struct QBook {
  float lo, hi;
  double scale;
};

__device__ __forceinline__ void minmax_block(float& mn, float& mx, float* smin, float* smax) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    mn = __builtin_fminf(mn, __shfl_xor(mn, d));
    mx = __builtin_fmaxf(mx, __shfl_xor(mx, d));
  }
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    smin[w] = mn;
    smax[w] = mx;
  }
  __syncthreads();
  mn = smin[0];
  mx = smax[0];
#pragma unroll
  for (int k = 1; k < kQThreads / kWave; ++k) {
    mn = __builtin_fminf(mn, smin[k]);
    mx = __builtin_fmaxf(mx, smax[k]);
  }
}

// Minimum and maximum of each kQChunk-element chunk of x.
// Grid: ceil(n / kQChunk) workgroups of kQThreads.
__global__ __launch_bounds__(kQThreads) void sdtw_u8_minmax_kernel(const float* __restrict__ x,
                                                                  int64_t n,
                                                                  float2* __restrict__ part) {
  __shared__ float smin[kQThreads / kWave], smax[kQThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kQChunk;
  float mn = inf_f32(), mx = -inf_f32();
#pragma unroll
  for (int u = 0; u < kQPer; ++u) {
    const int64_t i = base + threadIdx.x + u * kQThreads;
    if (i < n) {
      const float v = x[i];
      mn = __builtin_fminf(mn, v);
      mx = __builtin_fmaxf(mx, v);
    }
  }
  minmax_block(mn, mx, smin, smax);
  if (threadIdx.x == 0) part[blockIdx.x] = make_float2(mn, mx);
}

// The codebook from the chunk extremes.  One workgroup.
__global__ __launch_bounds__(kQThreads) void sdtw_u8_book_kernel(const float2* __restrict__ part,
                                                                int nparts,
                                                                QBook* __restrict__ book,
                                                                float* __restrict__ out) {
  __shared__ float smin[kQThreads / kWave], smax[kQThreads / kWave];
  float mn = inf_f32(), mx = -inf_f32();
  for (int i = threadIdx.x; i < nparts; i += kQThreads) {
    mn = __builtin_fminf(mn, part[i].x);
    mx = __builtin_fmaxf(mx, part[i].y);
  }
  minmax_block(mn, mx, smin, smax);
  if (threadIdx.x == 0) {
    const float lo = __builtin_fmaxf(mn, -kU8Clip);
    const float hi = __builtin_fminf(mx, kU8Clip);
    book->lo = lo;
    book->hi = hi;
    book->scale = hi > lo ? 255.0 / ((double)hi - (double)lo) : 0.0;
    out[0] = lo;
    out[1] = hi;
  }
}

// Codes of n packed values.  Grid-stride over elements.
__global__ __launch_bounds__(kQThreads) void sdtw_u8_encode_kernel(const float* __restrict__ x,
                                                                  int64_t n,
                                                                  const QBook* __restrict__ book,
                                                                  uint8_t* __restrict__ codes) {
  const double lo = book->lo;
  const double scale = book->scale;
  const int64_t stride = (int64_t)gridDim.x * kQThreads;
  for (int64_t i = (int64_t)blockIdx.x * kQThreads + threadIdx.x; i < n; i += stride) {
    double v = __builtin_rint(((double)x[i] - lo) * scale);
    v = v < 0.0 ? 0.0 : (v > 255.0 ? 255.0 : v);
    codes[i] = (uint8_t)(int)v;
  }
}

}  // namespace sdtw
