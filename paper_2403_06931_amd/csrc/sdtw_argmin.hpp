// sdtw_argmin.hpp -- reduction of the last DP row of a query to
// (cost, end_pos), and the small setup kernels.
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

// Exclusive prefix sum of the query lengths (offsets[0..batch]) in one
// workgroup: each thread sums a contiguous chunk, the chunk sums are scanned
// in LDS, then each thread writes its chunk's offsets.
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void sdtw_offsets_kernel(
    const int32_t* __restrict__ lens, int32_t batch, int64_t* __restrict__ offsets) {
  __shared__ int64_t s_sum[kScanThreads];
  const int tid = threadIdx.x;
  const int per = (batch + kScanThreads - 1) / kScanThreads;
  const int lo = min(batch, tid * per), hi = min(batch, lo + per);
  int64_t acc = 0;
  for (int i = lo; i < hi; ++i) acc += lens[i];
  s_sum[tid] = acc;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    const int64_t v = tid >= d ? s_sum[tid - d] : 0;
    __syncthreads();
    s_sum[tid] += v;
    __syncthreads();
  }
  int64_t run = s_sum[tid] - acc;                      // exclusive prefix of this chunk
  for (int i = lo; i < hi; ++i) {
    offsets[i] = run;
    run += lens[i];
  }
  if (tid == kScanThreads - 1) offsets[batch] = s_sum[tid];
}

// Processing order for the persistent form: queries sorted by the number
// of row passes they need (most first), so the longest work starts first and
// the short queries fill the tail.  Queries with equal pass counts are
// placed in an unspecified order; results do not depend on the order.  Also
// zeroes the work counter (a kernel, not a memset, so the sequence is safe to
// capture in a graph and replay).
constexpr int kOrderBins = 4096;

__global__ __launch_bounds__(kScanThreads) void sdtw_order_kernel(
    const int32_t* __restrict__ lens, int32_t batch, int32_t rows_per_pass,
    int32_t* __restrict__ order, int32_t* __restrict__ queue) {
  __shared__ int32_t s_cnt[kOrderBins];
  const int tid = threadIdx.x;
  for (int i = tid; i < kOrderBins; i += kScanThreads) s_cnt[i] = 0;
  if (tid == 0) queue[0] = 0;
  __syncthreads();
  for (int b = tid; b < batch; b += kScanThreads) {
    const int passes = min(kOrderBins - 1, (lens[b] + rows_per_pass - 1) / rows_per_pass);
    atomicAdd(&s_cnt[kOrderBins - 1 - passes], 1);     // descending by passes
  }
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int i = 0; i < kOrderBins; ++i) {
      const int c = s_cnt[i];
      s_cnt[i] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int b = tid; b < batch; b += kScanThreads) {
    const int passes = min(kOrderBins - 1, (lens[b] + rows_per_pass - 1) / rows_per_pass);
    const int at = atomicAdd(&s_cnt[kOrderBins - 1 - passes], 1);
    order[at] = b;
  }
}

}  // namespace sdtw
