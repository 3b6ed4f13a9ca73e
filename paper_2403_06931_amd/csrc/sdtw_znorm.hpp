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
//     with one wavefront each, the series held in registers (64 samples per
//     lane), both sums reduced within the wavefront with DPP moves: no
//     barrier and no LDS.  Loads and stores go through buffer resources
//     bounded by the series' length, so a lane needs no bounds test.  The
//     host passes the first element of every stride-th series in the kernel
//     arguments, so a wavefront finds its series by adding at most
//     stride - 1 lengths: no offset table and no extra launch.  Wavefronts
//     past those take the 4096-sample chunks of the long series, which the
//     host also lists in the arguments, and store each chunk's sum and sum of
//     squared deviations;
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
constexpr int kZWaveMax = kWave * kZWavePer;         // series standardised by one wavefront
constexpr int kZWavesPerWG = kZThreads / kWave;
constexpr int kZMaxLong = 32;                        // long series in the kernel arguments
constexpr int kZCoarse = 256;                        // prefix entries in the kernel arguments
constexpr int32_t kZDirectBatch = 16384;
constexpr int kZMaxStride = kZDirectBatch / kZCoarse;   // series per prefix entry, at most
static_assert(kZMaxStride <= kWave, "a wavefront sums the lengths after a prefix entry");
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
  int32_t stride;               // series per prefix entry
  int32_t nlong;                // long series
  int32_t long_chunks;          // their chunks
  ZLong lg[kZMaxLong];
  int64_t prefix[kZCoarse];     // first element of series k * stride
};

// 64-bit wavefront sums with DPP moves (no LDS traffic): pairs within quads,
// then mirrored half rows and rows of 16 lanes (all lanes of a group hold
// equal values by then, so a mirror adds the other half's sum), then the
// four row sums read out and added in row order.  The order is fixed, so the
// bits are the same on every run; every lane gets the result.
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long u) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffu), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xf, 0xf, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long u, int lane) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffu), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

template <typename T, typename Add>
__device__ __forceinline__ T wave_sum_dpp(T v, Add add) {
  auto bits = [](T x) { return __builtin_bit_cast(unsigned long long, x); };
  auto val = [](unsigned long long u) { return __builtin_bit_cast(T, u); };
  v = add(v, val(dpp_u64<0xb1>(bits(v))));   // quad_perm [1,0,3,2]
  v = add(v, val(dpp_u64<0x4e>(bits(v))));   // quad_perm [2,3,0,1]
  v = add(v, val(dpp_u64<0x141>(bits(v))));  // row_half_mirror
  v = add(v, val(dpp_u64<0x140>(bits(v))));  // row_mirror
  return add(add(add(val(readlane_u64(bits(v), 0)), val(readlane_u64(bits(v), 16))),
                 val(readlane_u64(bits(v), 32))),
             val(readlane_u64(bits(v), 48)));
}

__device__ __forceinline__ double wave_sum_f64(double v) {
  return wave_sum_dpp(v, [](double a, double b) { return a + b; });
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
  return wave_sum_dpp(v, [](long long a, long long b) { return a + b; });
}

// A buffer resource over m floats at p: loads past the end read zero and
// stores past it are dropped, so every lane loads and stores its 64 samples
// without a branch or a bounds test.  (The raw buffer builtins move 32-bit
// patterns: values are bit-cast, never converted.)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t znorm_rsrc(const float* p, int m) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, m * 4,
                                           0x00020000);
}

// The m (<= kZWaveMax) samples of a series or chunk, 64 per lane (sample
// lane + 64u in v[u]; zero past the end), all loads in flight together.
__device__ __forceinline__ void znorm_wave_load(__amdgpu_buffer_rsrc_t src, int lane,
                                                float (&v)[kZWavePer]) {
#pragma unroll
  for (int u = 0; u < kZWavePer; ++u)
    v[u] = __builtin_bit_cast(
        float, __builtin_amdgcn_raw_buffer_load_b32(src, (lane + kWave * u) * 4, 0, 0));
}

// Keep the samples as binary32 between passes: without this the compiler
// holds all 64 binary64 conversions live (128 more registers per lane).
__device__ __forceinline__ void znorm_fence(float (&v)[kZWavePer]) {
#pragma unroll
  for (int u = 0; u < kZWavePer; ++u) asm volatile("" : "+v"(v[u]));
}

// Sum of the m loaded samples and their sum of squared deviations from
// their mean, over the wavefront (four partial sums per lane, added in a
// fixed order).
__device__ __forceinline__ void znorm_wave_moments(float (&v)[kZWavePer], int m, int lane,
                                                   double& s1, double& m2) {
  double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < kZWavePer; ++u) a[u & 3] += (double)v[u];   // padding adds +0
  s1 = wave_sum_f64((a[0] + a[1]) + (a[2] + a[3]));
  znorm_fence(v);
  const double mk = s1 / m;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < kZWavePer; ++u) {
    const double d = (double)v[u] - mk;
    t[u & 3] += lane + kWave * u < m ? d * d : 0.0;
  }
  m2 = wave_sum_f64((t[0] + t[1]) + (t[2] + t[3]));
  znorm_fence(v);
}

__device__ __forceinline__ void znorm_wave_store(__amdgpu_buffer_rsrc_t dst, int lane,
                                                 const float (&v)[kZWavePer], double mean,
                                                 double sd) {
  const double inv = sd > 0.0 ? 1.0 / sd : 0.0;
#pragma unroll
  for (int u = 0; u < kZWavePer; ++u)
    __builtin_amdgcn_raw_buffer_store_b32(
        __builtin_bit_cast(uint32_t, (float)(((double)v[u] - mean) * inv)), dst,
        (lane + kWave * u) * 4, 0, 0);
}

// Long chunk c (0-based among all long chunks): its series descriptor and
// the chunk's place in the series.
__device__ __forceinline__ ZChunk znorm_long_chunk(const ZDirect& p, int c) {
  int j = 0;
  while (j + 1 < p.nlong && c >= p.lg[j + 1].c0) ++j;
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

// One wavefront per item: items [0, batch) are the series (a short one, of
// at most kZWaveMax samples, is standardised here; a long one's item does
// nothing), items [batch, batch + long_chunks) the chunks of the long series,
// which the host lists in the arguments: their sum and sum of squared
// deviations go to `part`.  A short series' first element is the prefix
// entry before it (host-given) plus at most stride - 1 lengths.  No barrier
// and no LDS: every wavefront works alone.
__global__ __launch_bounds__(kZThreads) void sdtw_znorm_direct_kernel(const ZDirect p) {
  const int lane = threadIdx.x & (kWave - 1);
  const int item = (int)blockIdx.x * kZWavesPerWG +
                   __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  float v[kZWavePer];
  if (item < p.batch) {
    const int b = item;
    const int e0 = (b / p.stride) * p.stride;   // series of the prefix entry
    const int n = __builtin_amdgcn_readfirstlane(p.lens[b]);
    const long long mine = lane < b - e0 ? (long long)p.lens[e0 + lane] : 0;
    if (n > kZWaveMax) return;                  // a long series: its chunks are elsewhere
    const int64_t off = p.prefix[b / p.stride] + wave_sum_i64(mine);
    znorm_wave_load(znorm_rsrc(p.x + off, n), lane, v);
    double s1, m2;
    znorm_wave_moments(v, n, lane, s1, m2);
    znorm_wave_store(znorm_rsrc(p.z + off, n), lane, v, s1 / n, __builtin_sqrt(m2 / n));
    return;
  }
  const int c = item - p.batch;
  if (c >= p.long_chunks) return;
  const ZChunk q = znorm_long_chunk(p, c);
  znorm_wave_load(znorm_rsrc(p.x + q.start, q.m), lane, v);
  double s1, m2;
  znorm_wave_moments(v, q.m, lane, s1, m2);
  if (lane == 0) {
    p.part[2 * (int64_t)c] = s1;
    p.part[2 * (int64_t)c + 1] = m2;
  }
}

// Long series: combine the series' chunk partials (each lane a fixed subset
// of the chunks in order, then the wavefront sum), then standardise this
// wavefront's chunk.  One wavefront per long chunk.
__global__ __launch_bounds__(kZThreads) void sdtw_znorm_long_apply_kernel(const ZDirect p) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = (int)blockIdx.x * kZWavesPerWG +
                __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  if (c >= p.long_chunks) return;
  const ZChunk q = znorm_long_chunk(p, c);
  float v[kZWavePer];
  znorm_wave_load(znorm_rsrc(p.x + q.start, q.m), lane, v);
  znorm_fence(v);
  double s = 0.0;
  for (int k = lane; k < q.nch; k += kWave) s += p.part[2 * (q.c0 + k)];
  const double mean = wave_sum_f64(s) / q.n;
  double t = 0.0;
  for (int k = lane; k < q.nch; k += kWave) {
    const int mk_n = min(kZChunk, q.n - k * kZChunk);
    const double d = p.part[2 * (q.c0 + k)] / mk_n - mean;
    t += p.part[2 * (q.c0 + k) + 1] + mk_n * (d * d);
  }
  const double sd = __builtin_sqrt(wave_sum_f64(t) / q.n);
  znorm_fence(v);
  znorm_wave_store(znorm_rsrc(p.z + q.start, q.m), lane, v, mean, sd);
}

}  // namespace sdtw
