// sdtw_bwd.hpp -- adjoint of the sDTW cost: walk-back gradient from column
// checkpoints.
//
// The cost of a query is the summed local cost along its optimal warp path,
// which the walk-back of Section 2 recovers from the end cell (N, end_pos) by
// repeatedly stepping to the cheapest of the cells (i-1,j-1), (i-1,j),
// (i,j-1) (ties: diagonal, then up, then left).  Away from ties the path is
// locally constant, so d cost / d q_i and d cost / d r_j are sums of the
// local-cost derivative over the path cells in row i / column j.
//
// The forward stored D(1..N, k*K) for every K-th column (K = ckpt_every), so
// every block of K columns can be recomputed on its own.  The backward runs
// in rounds, each covering the next G blocks of every unfinished query, from
// the block holding end_pos leftwards:
//
//   dirs   one wavefront per (query, block): recompute the block from its
//          left checkpoint and store a 2-bit direction code per cell to a
//          global scratch buffer (all blocks of the round in parallel);
//   walk   one wavefront per query: follow the codes from the current cell,
//          recording for every row the first and last column of the path in
//          that row; stop at row 1 or when the round's blocks are used up.
//
// A final kernel forms the gradients from the recorded rows: the path cells
// of one row are a run of columns and those of one column a run of rows, so
// every row sum and every column sum is an independent sequential sum, added
// in walk order (columns descending within a row, rows descending within a
// column).  Another kernel adds the per-query reference partials in
// increasing query order.
//
// Recompute mapping (the column-owning layout of the paper's Section 5.2
// kernel, which suits these narrow, tall blocks): lane l owns 16 adjacent
// reference columns of a 1024-column segment and walks down the rows, one row
// per step, one step behind lane l-1; lane l-1's right-most value reaches lane
// l through a DPP wave_shr:1 move, and so does the query value of the row.
// Each cell is recomputed with exactly the forward's operations, so the
// recomputed values and the directions taken from them are those of the
// full matrix.
#pragma once

#include "sdtw_common.hpp"

namespace sdtw {

constexpr int kDirCols = 16;                    // reference columns per lane
constexpr int kDirSeg = kWave * kDirCols;       // columns per segment
constexpr int kDirMaxRows = 8192;               // query + left column held in LDS
constexpr int kWalkChunk = 64;                  // code rows per walker LDS chunk
constexpr int kBwdMaxSlots = 8;                 // blocks per round per query

// Direction codes (2 bits per cell; cell c of a word at bits 2c, 2c+1).
constexpr uint32_t kDirDiag = 0;
constexpr uint32_t kDirUp = 1;
constexpr uint32_t kDirLeft = 2;

struct BwdParams {
  const float* queries;       // packed
  const int32_t* lens;        // [batch]
  const int64_t* offsets;     // [batch + 1]
  const float* reference;     // [ref_len]
  const float* grad_cost;     // [batch]
  const int64_t* end_pos;     // [batch]
  const float* ckpt;          // forward checkpoints (nullptr when n_ckpt == 0)
  float* grad_q;              // packed like queries
  float* ref_part;            // [batch][part_stride] per-query reference partials
  int32_t* path_lo;           // [batch] first reference column of the path
  int32_t* row_lo;            // packed like queries: first path column of each row
  int32_t* row_hi;            // packed like queries: last path column of each row
  int32_t* state;             // [batch][4]: current row (1-based), column, done
  uint32_t* codes;            // direction words, see code_segment()
  int64_t part_stride;
  int32_t batch;
  int32_t ref_len;
  int32_t ckpt_every;
  int32_t n_ckpt;
  int32_t nseg;               // segments per block, ceil(ckpt_every / kDirSeg)
  int32_t slots;              // blocks per round (G)
  int32_t max_rows;           // longest query (sizes the dirs kernel's LDS)
  int32_t round;
};

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t wave_uniform64(int64_t v) {
  const unsigned long long u = (unsigned long long)v;
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(u >> 32));
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(u & 0xffffffffu));
  return (int64_t)(((unsigned long long)hi << 32) | lo);
}

// Codes of segment s of round slot t of query b: n + 63 rows of 64 words;
// word l of row g holds the 16 codes of lane l at step g, i.e. of query row
// i = g - l + 1 and columns 16l .. 16l+15 of the segment.
__device__ __forceinline__ int64_t code_segment(const BwdParams& p, int b, int64_t qoff, int n,
                                                int t, int s) {
  const int64_t rows = (int64_t)n + kWave - 1;
  const int64_t base = (int64_t)p.slots * p.nseg * kWave * (qoff + (int64_t)(kWave - 1) * b);
  return base + ((int64_t)t * p.nseg + s) * rows * kWave;
}

// Local-cost derivative with respect to the query value at t = q - r.
template <int KIND>
__device__ __forceinline__ float dcost_dq(float q, float r) {
  const float t = q - r;
  if constexpr (KIND == kSquared) {
    return 2.0f * t;
  } else {
    return t > 0.0f ? 1.0f : (t < 0.0f ? -1.0f : 0.0f);
  }
}

// Walker state: start at (N, end_pos); row N's last path column is end_pos.
constexpr int kInitThreads = 256;

__global__ __launch_bounds__(kInitThreads) void sdtw_bwd_init_kernel(const BwdParams p) {
  const int b = blockIdx.x * kInitThreads + threadIdx.x;
  if (b >= p.batch) return;
  const int n = p.lens[b];
  const int e = (int)p.end_pos[b];
  p.state[4 * b + 0] = n;
  p.state[4 * b + 1] = e;
  p.state[4 * b + 2] = 0;
  p.state[4 * b + 3] = 0;
  p.row_hi[p.offsets[b] + n - 1] = e;
}

// One row step of the direction recompute.  MASKED: some lanes are outside
// rows 1..nrows and keep their state (row 0 before they start).
template <int KIND, bool MASKED>
__device__ __forceinline__ void dirs_step(int g, int lane, int nrows, const float* lq,
                                          float* ledge, const float (&rv)[kDirCols],
                                          float (&dprev)[kDirCols], float& last, float& shp,
                                          float& qv, uint32_t* __restrict__ out) {
  const int gi = g < nrows ? g : nrows - 1;
  const float shc = wave_shr1(ledge[gi], last);   // left neighbour on this row
  qv = wave_shr1(lq[gi], qv);                     // this row's query value
  float cur[kDirCols];
  uint32_t word = 0;
  float left = shc, diag = shp;
#pragma unroll
  for (int c = 0; c < kDirCols; ++c) {
    const float up = dprev[c];
    const float mn = min3(up, left, diag);
    const uint32_t code = diag == mn ? kDirDiag : (up == mn ? kDirUp : kDirLeft);
    word |= code << (2 * c);
    cur[c] = mn + local_cost<KIND>(qv, rv[c]);
    diag = up;
    left = cur[c];
  }
  out[(int64_t)g * kWave] = word;
  const int i = g - lane + 1;
  if (!MASKED || (i >= 1 && i <= nrows)) {
#pragma unroll
    for (int c = 0; c < kDirCols; ++c) dprev[c] = cur[c];
    last = cur[kDirCols - 1];
    // right column of this segment = left column of the next one; entry
    // i-1 was read by lane 0 at step i-1, 63 steps earlier
    if (lane == kWave - 1) ledge[i - 1] = last;
  }
  shp = shc;
}

// Recompute rows 1..i of one block (i = the walker's current row) and store
// its direction codes.  Grid: (batch, slots); one wavefront per workgroup.
// Dynamic LDS: query values and the left boundary column, 2 * max_rows floats.
template <int KIND>
__global__ __launch_bounds__(kWave) void sdtw_bwd_dirs_kernel(const BwdParams p) {
  extern __shared__ float dyn[];
  const int b = blockIdx.x;
  const int t = blockIdx.y;
  const int lane = threadIdx.x;
  if (wave_uniform(p.state[4 * b + 2]) != 0) return;
  const int K = p.ckpt_every;
  const int64_t e = wave_uniform64(p.end_pos[b]);
  const int blk_end = (int)(e / K);
  const int blk = blk_end - p.round * p.slots - t;
  if (blk < 0) return;
  const int n = wave_uniform(p.lens[b]);
  const int nrows = wave_uniform(p.state[4 * b + 0]);
  const int64_t qoff = wave_uniform64(p.offsets[b]);
  float* lq = dyn;
  float* ledge = dyn + p.max_rows;
  const float* __restrict__ q = p.queries + qoff;
  const float* ck = blk > 0 ? p.ckpt + qoff * p.n_ckpt + (int64_t)(blk - 1) * n : nullptr;
  for (int k = lane; k < nrows; k += kWave) {
    lq[k] = q[k];
    ledge[k] = blk > 0 ? ck[k] : inf_f32();
  }
  __syncthreads();

  const int bc0 = blk * K;
  const int bend = bc0 + K < p.ref_len ? bc0 + K : p.ref_len;
  int nseg = (bend - bc0 + kDirSeg - 1) / kDirSeg;
  if (blk == blk_end) nseg = (int)(e - bc0) / kDirSeg + 1;   // nothing right of end_pos
  for (int s = 0; s < nseg; ++s) {
    const int cs = bc0 + s * kDirSeg;
    float rv[kDirCols];
#pragma unroll
    for (int c = 0; c < kDirCols; ++c) {
      const int j = cs + lane * kDirCols + c;
      rv[c] = j < bend ? p.reference[j] : 0.0f;
    }
    uint32_t* out = p.codes + code_segment(p, b, qoff, n, t, s) + lane;
    float dprev[kDirCols];
#pragma unroll
    for (int c = 0; c < kDirCols; ++c) dprev[c] = 0.0f;      // row 0
    float last = 0.0f, shp = 0.0f, qv = 0.0f;
    const int g_end = nrows + kWave - 1;
    const int g_head = g_end < kWave - 1 ? g_end : kWave - 1;
    int g = 0;
    for (; g < g_head; ++g)
      dirs_step<KIND, true>(g, lane, nrows, lq, ledge, rv, dprev, last, shp, qv, out);
    for (; g < nrows; ++g)
      dirs_step<KIND, false>(g, lane, nrows, lq, ledge, rv, dprev, last, shp, qv, out);
    for (; g < g_end; ++g)
      dirs_step<KIND, true>(g, lane, nrows, lq, ledge, rv, dprev, last, shp, qv, out);
  }
}

// Follow the direction codes of this round's blocks.  Grid: batch; one
// wavefront per workgroup; every lane runs the same (uniform) walk and lane
// 0 stores.  Code rows are staged through LDS 64 at a time: within a
// segment the code row g = i - 1 + (lane owning column j) never increases
// along the walk.
__global__ __launch_bounds__(kWave) void sdtw_bwd_walk_kernel(const BwdParams p) {
  __shared__ uint32_t chunk[kWalkChunk * kWave];
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  if (wave_uniform(p.state[4 * b + 2]) != 0) return;
  int i = wave_uniform(p.state[4 * b + 0]);
  int j = wave_uniform(p.state[4 * b + 1]);
  const int n = wave_uniform(p.lens[b]);
  const int64_t qoff = wave_uniform64(p.offsets[b]);
  const int K = p.ckpt_every;
  const int blk_end = (int)(wave_uniform64(p.end_pos[b]) / K);
  int32_t* rlo = p.row_lo + qoff - 1;           // indexed by 1-based row
  int32_t* rhi = p.row_hi + qoff - 1;
  const int code_rows = n + kWave - 1;
  int done = 0;

  for (int t = 0; t < p.slots && !done; ++t) {
    const int blk = blk_end - p.round * p.slots - t;
    if (blk < 0) break;
    const int bc0 = blk * K;
    for (int s = (j - bc0) / kDirSeg; s >= 0 && !done; --s) {
      const int cs = bc0 + s * kDirSeg;
      const uint32_t* seg = p.codes + code_segment(p, b, qoff, n, t, s);
      int kc = -1;                              // code chunk held in LDS
      while (j >= cs) {
        const int L = (j - cs) >> 4;
        const int c = (j - cs) & (kDirCols - 1);
        const int g = i - 1 + L;
        const int k = g / kWalkChunk;
        if (k != kc) {
          // stage code rows [64k, 64k + 64); rows past the segment's end
          // are never addressed
          __builtin_amdgcn_wave_barrier();
          for (int m = 0; m < kWalkChunk; ++m) {
            const int row = k * kWalkChunk + m;
            if (row < code_rows) chunk[m * kWave + lane] = seg[(int64_t)row * kWave + lane];
          }
          __builtin_amdgcn_wave_barrier();
          kc = k;
        }
        const uint32_t w =
            (uint32_t)wave_uniform((int)chunk[(g - k * kWalkChunk) * kWave + L]);
        // pass through the cells c, c-1, ... of this word whose code is
        // "left"; the first other one ends the run in this row
        const uint32_t is_left = (w >> 1) & ~w & 0x55555555u;
        const uint32_t upto = c == kDirCols - 1 ? 0xffffffffu : ((1u << (2 * c + 2)) - 1u);
        const uint32_t stop = ~is_left & 0x55555555u & upto;
        if (stop == 0) {
          j -= c + 1;                           // into the previous lane's columns
          continue;
        }
        const int bit = 31 - __builtin_clz(stop);
        j -= c - (bit >> 1);
        if (i == 1) {                           // the start cell
          if (lane == 0) {
            rlo[1] = j;
            p.path_lo[b] = j;
          }
          done = 1;
          break;
        }
        const uint32_t code = (w >> bit) & 3u;
        if (lane == 0) rlo[i] = j;
        i -= 1;
        if (code == kDirDiag) j -= 1;
        if (lane == 0) rhi[i] = j;
      }
    }
  }
  if (lane == 0) {
    p.state[4 * b + 0] = i;
    p.state[4 * b + 1] = j;
    p.state[4 * b + 2] = done;
  }
}

// Gradients from the recorded path rows.  Grid: batch; kGradThreads threads.
//   grad_q[i]      = sum over the row's path columns j (descending) of g*dc/dq
//   ref_part[b][j] = sum over the column's path rows i (descending) of -g*dc/dq
// for j in [path_lo, end_pos].  Row i's columns are [row_lo[i], row_hi[i]];
// both bounds are nondecreasing in i, so column j's rows are found by binary
// search.
constexpr int kGradThreads = 256;

template <int KIND>
__global__ __launch_bounds__(kGradThreads) void sdtw_bwd_grad_kernel(const BwdParams p) {
  const int b = blockIdx.x;
  const int n = p.lens[b];
  const int64_t qoff = p.offsets[b];
  const float* __restrict__ q = p.queries + qoff;
  const float* __restrict__ r = p.reference;
  const int32_t* __restrict__ rlo = p.row_lo + qoff - 1;
  const int32_t* __restrict__ rhi = p.row_hi + qoff - 1;
  const float gcost = p.grad_cost[b];
  float* __restrict__ gq = p.grad_q + qoff;
  float* __restrict__ part = p.ref_part + (int64_t)b * p.part_stride;

  // (the clamps only keep every access in bounds; a finished walk records
  // every row, with columns in [0, end_pos])
  const int jhi = (int)p.end_pos[b];
  for (int i = 1 + (int)threadIdx.x; i <= n; i += kGradThreads) {
    const float qi = q[i - 1];
    const int lo = rlo[i] > 0 ? rlo[i] : 0;
    const int hi = rhi[i] < jhi ? rhi[i] : jhi;
    float acc = 0.0f;
    for (int jj = hi; jj >= lo; --jj) acc = acc + gcost * dcost_dq<KIND>(qi, r[jj]);
    gq[i - 1] = acc;
  }

  const int jlo = p.path_lo[b] > 0 ? p.path_lo[b] : 0;
  for (int jj = jlo + (int)threadIdx.x; jj <= jhi; jj += kGradThreads) {
    int a = 1, z = n;                           // first row whose last column reaches jj
    while (a < z) {
      const int mid = (a + z) >> 1;
      if (rhi[mid] >= jj) z = mid; else a = mid + 1;
    }
    const int top = a;
    z = n;                                      // last row whose first column is <= jj
    while (a < z) {
      const int mid = (a + z + 1) >> 1;
      if (rlo[mid] <= jj) a = mid; else z = mid - 1;
    }
    const int bottom = a;
    const float rj = r[jj];
    float acc = 0.0f;
    for (int ii = bottom; ii >= top; --ii)
      acc = acc + (-(gcost * dcost_dq<KIND>(q[ii - 1], rj)));
    part[jj] = acc;
  }
}

// grad_reference[j] = sum over queries b (increasing) whose path covers
// column j of ref_part[b][j]; +0 where no path passes.
constexpr int kRefReduceThreads = 256;

__global__ __launch_bounds__(kRefReduceThreads) void sdtw_ref_reduce_kernel(
    const float* __restrict__ ref_part, int64_t part_stride, const int32_t* __restrict__ lo,
    const int64_t* __restrict__ hi, int32_t batch, int32_t ref_len, float* __restrict__ grad_ref) {
  const int j = blockIdx.x * kRefReduceThreads + threadIdx.x;
  if (j >= ref_len) return;
  float acc = 0.0f;
  for (int b = 0; b < batch; ++b) {
    if (j >= lo[b] && j <= (int)hi[b]) acc = acc + ref_part[(int64_t)b * part_stride + j];
  }
  grad_ref[j] = acc;
}

}  // namespace sdtw
