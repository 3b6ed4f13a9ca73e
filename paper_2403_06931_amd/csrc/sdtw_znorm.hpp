// sdtw_znorm.hpp -- batch z-normalisation, the step before the DP (the
// paper's normaliser, Section 5.1 "Normalizer implementation", standardisation
// equation): every series of a packed batch becomes z = (x - mean) / S with S
// the population standard deviation.  Included by the API translation unit
// only.
//
// Statistics are reduced in binary64 in a fixed order, so results do not
// depend on scheduling; z = (x - mean) * (1/S) is formed in binary64 (one
// reciprocal per series instead of a division per sample) and rounded once to
// binary32.  The data are read once and written once wherever a series fits
// on one compute unit; that traffic (8 bytes per sample) is the bound.
//
// Direct form (batches of up to kZDirectBatch series with at most kZMaxLong
// series longer than kZWaveMax):
//   * one launch standardises every short series (up to kZWaveMax samples)
//     with one wavefront each, the series held in registers (up to 64 per
//     lane, loads coalesced across the wavefront) and both sums reduced by a
//     butterfly within the wavefront: no barrier and no LDS.  A workgroup
//     takes kZSeriesPerWG consecutive series and finds where they start by
//     summing the lengths before them (a few kilobytes from L2), so no
//     offset table and no extra launch is needed.  Workgroups past those
//     take the chunks of the long series, which the host describes in the
//     kernel arguments (it knows their offsets from the host lengths), and
//     store each chunk's sum and sum of squared deviations;
//   * a second launch, only when there are long series, combines a long
//     series' chunk partials exactly in a fixed order (sum of squares = sum
//     over chunks of the chunk's own sum plus n_k (mean_k - mean)^2) and
//     standardises each chunk after reading it once more.
// Table form (any batch): a one-workgroup index kernel builds element and
// chunk offsets and the chunk -> series map, one workgroup per chunk of
// kZChunk samples computes the chunk statistics (and finishes single-chunk
// series), and the same combine-and-standardise step finishes the rest.
#pragma once

#include "sdtw_common.hpp"
#include "sdtw_setup.hpp"

namespace sdtw {

constexpr int kZThreads = 256;                  // 4 wavefronts
constexpr int kZPer = 16;                       // elements per thread
constexpr int kZChunk = kZThreads * kZPer;      // elements per workgroup

struct ZParams {
  const float* x;               // packed input series
  float* z;                     // packed output (may equal x)
  const int32_t* lens;          // [batch]
  const int64_t* offsets;       // [batch + 1] first element of each series
  const int64_t* chunk_off;     // [batch + 1] first chunk of each series
  const int32_t* chunk_series;  // [chunks] series of each chunk
  double* part;                 // [chunks][2] chunk sum, chunk sum of squared deviations
  int32_t batch;
};

__host__ __device__ constexpr int64_t znorm_chunks_of(int64_t n) {
  return (n + kZChunk - 1) / kZChunk;
}

// Element and chunk offsets of every series and the series of every chunk,
// in one workgroup (the scan of sdtw_offsets_kernel, over two quantities).
// A thread maps the first kZOwnChunks chunks of its own series; the rest of
// a longer series (a reference) is mapped by the whole workgroup.
constexpr int kZOwnChunks = 8;
constexpr int kZLongMax = 256;                  // long series listed in LDS

__global__ __launch_bounds__(kScanThreads) void sdtw_znorm_index_kernel(
    const int32_t* __restrict__ lens, int32_t batch, int64_t* __restrict__ offsets,
    int64_t* __restrict__ chunk_off, int32_t* __restrict__ chunk_series) {
  __shared__ int64_t s_el[kScanThreads];
  __shared__ int64_t s_ch[kScanThreads];
  __shared__ int32_t s_long[kZLongMax];
  __shared__ int64_t s_long_c0[kZLongMax];
  __shared__ int32_t s_nlong;
  const int tid = threadIdx.x;
  if (tid == 0) s_nlong = 0;
  const int per = (batch + kScanThreads - 1) / kScanThreads;
  const int lo = min(batch, tid * per), hi = min(batch, lo + per);
  int64_t el = 0, ch = 0;
  for (int i = lo; i < hi; ++i) {
    el += lens[i];
    ch += znorm_chunks_of(lens[i]);
  }
  s_el[tid] = el;
  s_ch[tid] = ch;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    const int64_t a = tid >= d ? s_el[tid - d] : 0;
    const int64_t c = tid >= d ? s_ch[tid - d] : 0;
    __syncthreads();
    s_el[tid] += a;
    s_ch[tid] += c;
    __syncthreads();
  }
  int64_t re = s_el[tid] - el, rc = s_ch[tid] - ch;
  for (int i = lo; i < hi; ++i) {
    offsets[i] = re;
    chunk_off[i] = rc;
    const int64_t nc = znorm_chunks_of(lens[i]);
    const int64_t own = nc < kZOwnChunks ? nc : kZOwnChunks;
    for (int64_t k = 0; k < own; ++k) chunk_series[rc + k] = i;
    if (nc > own) {
      const int slot = atomicAdd(&s_nlong, 1);
      if (slot < kZLongMax) {
        s_long[slot] = i;
        s_long_c0[slot] = rc;
      } else {
        for (int64_t k = own; k < nc; ++k) chunk_series[rc + k] = i;
      }
    }
    re += lens[i];
    rc += nc;
  }
  if (tid == kScanThreads - 1) {
    offsets[batch] = s_el[tid];
    chunk_off[batch] = s_ch[tid];
  }
  __syncthreads();
  const int nlong = s_nlong < kZLongMax ? s_nlong : kZLongMax;
  for (int t = 0; t < nlong; ++t) {
    const int i = s_long[t];
    const int64_t c0 = s_long_c0[t];
    const int64_t nc = znorm_chunks_of(lens[i]);
    for (int64_t k = kZOwnChunks + tid; k < nc; k += kScanThreads) chunk_series[c0 + k] = i;
  }
}

// Sum over the workgroup in a fixed order: a butterfly within each
// wavefront (every lane ends with the same bits, since each step adds the
// same two values), then the wavefront sums in index order.
__device__ __forceinline__ double znorm_block_sum(double v, double* red) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int w = 1; w < kZThreads / kWave; ++w) s += red[w];
  __syncthreads();                              // red is reused by the next call
  return s;
}

struct ZChunk {
  int b, n, k, nch, m;          // series, its length, chunk index, chunks, elements here
  int64_t c0, start;            // series' first chunk, first element of this chunk
};

__device__ __forceinline__ ZChunk znorm_chunk(const ZParams& p, int c) {
  ZChunk q;
  q.b = p.chunk_series[c];
  q.n = p.lens[q.b];
  q.c0 = p.chunk_off[q.b];
  q.nch = (int)(p.chunk_off[q.b + 1] - q.c0);
  q.k = (int)(c - q.c0);
  q.start = p.offsets[q.b] + (int64_t)q.k * kZChunk;
  q.m = min(kZChunk, q.n - q.k * kZChunk);
  return q;
}

__device__ __forceinline__ void znorm_load(const ZParams& p, const ZChunk& q, float (&v)[kZPer]) {
#pragma unroll
  for (int u = 0; u < kZPer; ++u) {
    const int i = threadIdx.x + u * kZThreads;
    v[u] = i < q.m ? p.x[q.start + i] : 0.0f;
  }
}

__device__ __forceinline__ void znorm_store(const ZParams& p, const ZChunk& q,
                                            const float (&v)[kZPer], double mean, double s) {
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
#pragma unroll
  for (int u = 0; u < kZPer; ++u) {
    const int i = threadIdx.x + u * kZThreads;
    if (i < q.m) p.z[q.start + i] = (float)(((double)v[u] - mean) * inv);
  }
}

// Chunk statistics; series of one chunk are standardised here.
// Grid: one workgroup per chunk.
__global__ __launch_bounds__(kZThreads) void sdtw_znorm_stats_kernel(const ZParams p) {
  __shared__ double red[kZThreads / kWave];
  const ZChunk q = znorm_chunk(p, blockIdx.x);
  float v[kZPer];
  znorm_load(p, q, v);
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kZPer; ++u) s += (double)v[u];     // padding adds +0
  const double s1 = znorm_block_sum(s, red);
  const double mk = s1 / q.m;
  double t = 0.0;
#pragma unroll
  for (int u = 0; u < kZPer; ++u) {
    if (threadIdx.x + u * kZThreads < q.m) {
      const double d = (double)v[u] - mk;
      t += d * d;
    }
  }
  const double m2 = znorm_block_sum(t, red);
  if (q.nch == 1) {
    znorm_store(p, q, v, mk, __builtin_sqrt(m2 / q.n));
  } else if (threadIdx.x == 0) {
    p.part[2 * (int64_t)blockIdx.x] = s1;
    p.part[2 * (int64_t)blockIdx.x + 1] = m2;
  }
}

// Series of several chunks: combine the chunk partials, then standardise
// this workgroup's chunk.  Grid: one workgroup per chunk.
__global__ __launch_bounds__(kZThreads) void sdtw_znorm_apply_kernel(const ZParams p) {
  __shared__ double red[kZThreads / kWave];
  const ZChunk q = znorm_chunk(p, blockIdx.x);
  if (q.nch == 1) return;
  double s = 0.0;
  for (int k = threadIdx.x; k < q.nch; k += kZThreads) s += p.part[2 * (q.c0 + k)];
  const double mean = znorm_block_sum(s, red) / q.n;
  double t = 0.0;
  for (int k = threadIdx.x; k < q.nch; k += kZThreads) {
    const int mk_n = min(kZChunk, q.n - k * kZChunk);
    const double d = p.part[2 * (q.c0 + k)] / mk_n - mean;
    t += p.part[2 * (q.c0 + k) + 1] + mk_n * (d * d);
  }
  const double sd = __builtin_sqrt(znorm_block_sum(t, red) / q.n);
  float v[kZPer];
  znorm_load(p, q, v);
  znorm_store(p, q, v, mean, sd);
}

// ------------------------------------------------------------ direct form

constexpr int kZWavePer = 64;                        // samples per lane
constexpr int kZWaveMax = kWave * kZWavePer;         // series standardised by one wave
constexpr int kZSeriesPerWG = kZThreads / kWave;     // one wave per series
constexpr int kZMaxLong = 32;                        // long series in the kernel arguments
constexpr int32_t kZDirectBatch = 16384;
static_assert(kZWaveMax == kZChunk, "a short series is one chunk of the table form");

struct ZLong {
  int64_t off;                  // first element of the series
  int32_t b, n;                 // series index and length
  int32_t c0, nch;              // its first chunk among the long chunks, chunk count
};

struct ZDirect {
  const float* x;
  float* z;
  const int32_t* lens;
  double* part;                 // [long chunks][2]
  int32_t batch;
  int32_t short_wgs;            // workgroups of the short series (first in the grid)
  int32_t nlong;
  ZLong lg[kZMaxLong];
};

// Sum over the 64 lanes of a wavefront: every lane ends with the same bits
// (each step adds the same two values, and binary64 addition commutes).
__device__ __forceinline__ double znorm_wave_sum(double v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

// Long chunk c (0-based among all long chunks): its series descriptor and
// the chunk's place in the series.
__device__ __forceinline__ ZChunk znorm_long_chunk(const ZDirect& p, int c, int* lg_index) {
  int j = 0;
  while (j + 1 < p.nlong && c >= p.lg[j + 1].c0) ++j;
  *lg_index = j;
  const ZLong L = p.lg[j];
  ZChunk q;
  q.b = L.b;
  q.n = L.n;
  q.c0 = L.c0;
  q.nch = L.nch;
  q.k = c - L.c0;
  q.start = L.off + (int64_t)q.k * kZChunk;
  q.m = min(kZChunk, q.n - q.k * kZChunk);
  return q;
}

__device__ __forceinline__ void znorm_chunk_load(const float* x, const ZChunk& q,
                                                 float (&v)[kZPer]) {
#pragma unroll
  for (int u = 0; u < kZPer; ++u) {
    const int i = threadIdx.x + u * kZThreads;
    v[u] = i < q.m ? x[q.start + i] : 0.0f;
  }
}

// Short series: one wave each; long-series chunks: their partials.
__global__ __launch_bounds__(kZThreads) void sdtw_znorm_direct_kernel(const ZDirect p) {
  __shared__ double red[kZThreads / kWave];
  if ((int)blockIdx.x >= p.short_wgs) {
    int j;
    const ZChunk q = znorm_long_chunk(p, (int)blockIdx.x - p.short_wgs, &j);
    float v[kZPer];
    znorm_chunk_load(p.x, q, v);
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kZPer; ++u) s += (double)v[u];   // padding adds +0
    const double s1 = znorm_block_sum(s, red);
    const double mk = s1 / q.m;
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < kZPer; ++u) {
      if (threadIdx.x + u * kZThreads < q.m) {
        const double d = (double)v[u] - mk;
        t += d * d;
      }
    }
    const double m2 = znorm_block_sum(t, red);
    if (threadIdx.x == 0) {
      const int64_t c = (int64_t)blockIdx.x - p.short_wgs;
      p.part[2 * c] = s1;
      p.part[2 * c + 1] = m2;
    }
    return;
  }
  // where this workgroup's first series starts: the lengths before it
  __shared__ unsigned long long s_pre;
  const int first = (int)blockIdx.x * kZSeriesPerWG;
  if (threadIdx.x == 0) s_pre = 0;
  __syncthreads();
  unsigned long long acc = 0;
  for (int k = threadIdx.x; k < first; k += kZThreads) acc += (unsigned long long)p.lens[k];
  atomicAdd(&s_pre, acc);
  __syncthreads();
  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int b = first + wv;
  if (b >= p.batch) return;                     // no barrier below
  int64_t off = (int64_t)s_pre;
  for (int k = first; k < b; ++k) off += p.lens[k];
  const int n = p.lens[b];
  if (n > kZWaveMax) return;                    // a long series: its chunks are elsewhere
  const int nu = (n + kWave - 1) / kWave;       // loads per lane (uniform)
  const float* __restrict__ x = p.x + off;
  float v[kZWavePer];
#pragma unroll
  for (int u = 0; u < kZWavePer; ++u) {
    const int i = lane + u * kWave;
    v[u] = (u < nu && i < n) ? x[i] : 0.0f;
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kZWavePer; ++u) s += (double)v[u];   // padding adds +0
  const double mean = znorm_wave_sum(s) / n;
  double t = 0.0;
#pragma unroll
  for (int u = 0; u < kZWavePer; ++u) {
    if (lane + u * kWave < n) {
      const double d = (double)v[u] - mean;
      t += d * d;
    }
  }
  const double sd = __builtin_sqrt(znorm_wave_sum(t) / n);
  const double inv = sd > 0.0 ? 1.0 / sd : 0.0;
  float* __restrict__ z = p.z + off;
#pragma unroll
  for (int u = 0; u < kZWavePer; ++u) {
    const int i = lane + u * kWave;
    if (u < nu && i < n) z[i] = (float)(((double)v[u] - mean) * inv);
  }
}

// Long series: combine the chunk partials (fixed order), standardise the
// chunk.  Grid: one workgroup per long chunk.
__global__ __launch_bounds__(kZThreads) void sdtw_znorm_long_apply_kernel(const ZDirect p) {
  __shared__ double red[kZThreads / kWave];
  int j;
  const ZChunk q = znorm_long_chunk(p, (int)blockIdx.x, &j);
  double s = 0.0;
  for (int k = threadIdx.x; k < q.nch; k += kZThreads) s += p.part[2 * (q.c0 + k)];
  const double mean = znorm_block_sum(s, red) / q.n;
  double t = 0.0;
  for (int k = threadIdx.x; k < q.nch; k += kZThreads) {
    const int mk_n = min(kZChunk, q.n - k * kZChunk);
    const double d = p.part[2 * (q.c0 + k)] / mk_n - mean;
    t += p.part[2 * (q.c0 + k) + 1] + mk_n * (d * d);
  }
  const double sd = __builtin_sqrt(znorm_block_sum(t, red) / q.n);
  float v[kZPer];
  znorm_chunk_load(p.x, q, v);
  const double inv = sd > 0.0 ? 1.0 / sd : 0.0;
#pragma unroll
  for (int u = 0; u < kZPer; ++u) {
    const int i = threadIdx.x + u * kZThreads;
    if (i < q.m) p.z[q.start + i] = (float)(((double)v[u] - mean) * inv);
  }
}

}  // namespace sdtw
