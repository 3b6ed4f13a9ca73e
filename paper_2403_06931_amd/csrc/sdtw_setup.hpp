// sdtw_setup.hpp -- small one-workgroup kernels that run before the DP
// kernels: the query offset table and the processing order of the
// persistent form.  Included by the API translation unit only.
#pragma once

#include "sdtw_common.hpp"

namespace sdtw {

// Exclusive prefix sum of the query lengths (offsets[0..batch]) in one
// workgroup: each thread sums a contiguous chunk, the chunk sums are scanned
// in LDS, then each thread writes its chunk's offsets.  With ranks != nullptr
// it also writes, per query, the number of earlier queries longer than
// `rows` (the row-buffer slot of a query that needs several row passes).
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void sdtw_offsets_kernel(
    const int32_t* __restrict__ lens, int32_t batch, int64_t* __restrict__ offsets,
    int32_t rows, int32_t* __restrict__ ranks) {
  __shared__ int64_t s_sum[kScanThreads];
  __shared__ int32_t s_cnt[kScanThreads];
  const int tid = threadIdx.x;
  const int per = (batch + kScanThreads - 1) / kScanThreads;
  const int lo = min(batch, tid * per), hi = min(batch, lo + per);
  int64_t acc = 0;
  int32_t cnt = 0;
  for (int i = lo; i < hi; ++i) {
    acc += lens[i];
    cnt += lens[i] > rows ? 1 : 0;
  }
  s_sum[tid] = acc;
  s_cnt[tid] = cnt;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    const int64_t v = tid >= d ? s_sum[tid - d] : 0;
    const int32_t c = tid >= d ? s_cnt[tid - d] : 0;
    __syncthreads();
    s_sum[tid] += v;
    s_cnt[tid] += c;
    __syncthreads();
  }
  int64_t run = s_sum[tid] - acc;                      // exclusive prefix of this chunk
  int32_t rank = s_cnt[tid] - cnt;
  for (int i = lo; i < hi; ++i) {
    offsets[i] = run;
    run += lens[i];
    if (ranks != nullptr) {
      ranks[i] = rank;
      rank += lens[i] > rows ? 1 : 0;
    }
  }
  if (tid == kScanThreads - 1) offsets[batch] = s_sum[tid];
}

// Processing order for the persistent form: queries sorted by their work
// (most first), so the longest work starts first and the short queries fill
// the tail.  Work is counted in quarter passes: the full passes, then the
// last pass in the form the kernel runs it, a quarter, half or
// three-quarter pass when its rows fit and the tile has that form
// (min_quarters = 1: all three, 2: the half pass only, 4: none), else a
// whole pass.  (Counting every last pass as a whole one left the modelled
// makespan of the 4,096 x U{250..4,000} batch 8.6 % above the balanced one,
// against 2-3 % this way.)  Queries with equal work are placed in an
// unspecified order; results do not depend on the order.  Also zeroes the work counter (a kernel, not a memset, so the
// sequence is safe to capture in a graph and replay).
constexpr int kOrderBins = 4096;

__device__ __forceinline__ int order_key(int n, int rows, int min_quarters) {
  const int full = n > 0 ? (n - 1) / rows : 0;
  const int left = n - full * rows;
  int last = 4;
  if (min_quarters <= 1 && left <= 3 * rows / 4) last = 3;
  if (min_quarters <= 2 && left <= rows / 2) last = 2;
  if (min_quarters <= 1 && left <= rows / 4) last = 1;
  return min(kOrderBins - 1, 4 * full + last);
}

__global__ __launch_bounds__(kScanThreads) void sdtw_order_kernel(
    const int32_t* __restrict__ lens, int32_t batch, int32_t rows_per_pass,
    int32_t min_quarters, int32_t* __restrict__ order, int32_t* __restrict__ queue) {
  __shared__ int32_t s_cnt[kOrderBins];
  const int tid = threadIdx.x;
  for (int i = tid; i < kOrderBins; i += kScanThreads) s_cnt[i] = 0;
  if (tid == 0) queue[0] = 0;
  __syncthreads();
  for (int b = tid; b < batch; b += kScanThreads) {
    const int key = order_key(lens[b], rows_per_pass, min_quarters);
    atomicAdd(&s_cnt[kOrderBins - 1 - key], 1);        // descending by work
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
    const int key = order_key(lens[b], rows_per_pass, min_quarters);
    const int at = atomicAdd(&s_cnt[kOrderBins - 1 - key], 1);
    order[at] = b;
  }
}

}  // namespace sdtw
