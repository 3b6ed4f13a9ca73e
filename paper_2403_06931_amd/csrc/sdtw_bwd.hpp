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
// Memory: the forward stored D(1..N, k*K) for every K-th column (K =
// ckpt_every).  One workgroup per query walks its path block by block, from
// the block holding end_pos leftwards, without ever holding the N x M matrix:
//
//   phase 1  recompute the block from its left checkpoint, rows 1..i (i the
//            path's current row), keeping only the last column of every
//            S-column segment (global scratch);
//   phase 2  for each segment the path enters, right to left: recompute it
//            from its left column, writing a 2-bit direction code per cell
//            into LDS (S x rows fits in 128 KiB), then wave 0 walks it.
//
// The recompute uses the column-owning mapping of the paper's Section 5.2
// kernel, which suits these narrow, tall segments: lane L owns 4 adjacent
// reference columns and walks down the rows, one row per step, one step
// behind lane L-1; a lane's right-most value reaches lane L+1 through a DPP
// wave_shr:1 move, and wave w's lane 63 hands it to wave w+1 through an LDS
// ring (one barrier every KSTEP steps, wave w+1 lagging by KSTEP-1 extra
// steps, as in the forward kernel).  Each cell is recomputed with exactly the
// forward's operations, so the recomputed values are bit-identical.
//
// Gradient accumulation (matches the walk order of the definition in
// include/sdtw.h): the walker keeps the running sum of the current row
// (query gradient) and of the current column (per-query reference partial)
// and stores each when the path leaves that row / column.  A second kernel
// adds the per-query reference partials in increasing query order.
#pragma once

#include "sdtw_common.hpp"

namespace sdtw {

struct BwdParams {
  const float* queries;       // packed
  const int32_t* lens;        // [batch]
  const int64_t* offsets;     // [batch + 1] or nullptr (summed in-kernel)
  const float* reference;     // [ref_len]
  const float* grad_cost;     // [batch]
  const int64_t* end_pos;     // [batch]
  const float* ckpt;          // forward checkpoints (may be nullptr if n_ckpt == 0)
  float* grad_q;              // packed like queries
  float* ref_part;            // [batch][part_stride] per-query reference partials
  int32_t* path_lo;           // [batch] first reference column of the path
  float* colbuf;              // segment boundary columns: query b at offset(b) * seg_per_block
  int64_t part_stride;
  int32_t batch;
  int32_t ref_len;
  int32_t ckpt_every;
  int32_t n_ckpt;
  int32_t seg_per_block;      // ceil(ckpt_every / S)
};

constexpr int kBwdCols = 4;                 // reference columns per lane
constexpr int kBwdDirBytes = 131072;        // LDS for direction codes
constexpr int kBwdStepsPerBarrier = 8;

template <int W>
struct BwdShape {
  static constexpr int THREADS = kWave * W;
  static constexpr int S = THREADS * kBwdCols;              // segment width (columns)
  static constexpr int MAX_ROWS = kBwdDirBytes / THREADS;   // one byte per lane per row
  static constexpr int KSTEP = kBwdStepsPerBarrier;
  static constexpr int LAG = KSTEP - 1;
  static constexpr int SH = 2 * KSTEP;                      // handoff ring (rows)
};

// Direction codes (2 bits).
constexpr int kDirDiag = 0;
constexpr int kDirUp = 1;
constexpr int kDirLeft = 2;

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Shared memory of the backward kernel.
template <int W>
struct BwdSmem {
  using S = BwdShape<W>;
  uint8_t dirs[kBwdDirBytes];                 // [row - 1][lane]: 4 codes, 2 bits each
  float q[S::MAX_ROWS];                       // this query's values
  float left[S::MAX_ROWS];                    // left boundary column of the segment
  float rseg[S::S];                           // reference values of the segment
  float ring[W][S::SH];                       // wave -> wave handoff of the right edge
  int state[4];                               // walker -> team: i, j, done
};

// Recompute rows 1..nrows of the segment [c0, c0 + ncols) (ncols <= S).
// Inputs in LDS: sm.q (query), sm.left (D(i, c0-1), i = 1..nrows; +inf when
// c0 is the first column of the reference), sm.rseg (reference values, zero
// past the segment).  Row 0 is the free-start zero row.
// DIRS: write each cell's direction code to sm.dirs.
// RIGHT: write D(i, c0 + S - 1) to right[i - 1] (full segments only).
template <int W, int KIND, bool DIRS, bool RIGHT>
__device__ __forceinline__ void seg_dp(BwdSmem<W>& sm, int nrows, float* __restrict__ right) {
  using S = BwdShape<W>;
  constexpr int C = kBwdCols, KSTEP = S::KSTEP, LAG = S::LAG, SH = S::SH;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = wave_uniform(tid / kWave);
  const int pos = wave * kWave + lane;
  const int delay = pos + wave * LAG;
  const int lane0_delay = wave * (kWave + LAG);
  const int lane63_delay = lane0_delay + kWave - 1;

  float rv[C];
#pragma unroll
  for (int c = 0; c < C; ++c) rv[c] = sm.rseg[pos * C + c];
  float dprev[C];                               // row i-1 of this lane's columns
#pragma unroll
  for (int c = 0; c < C; ++c) dprev[c] = 0.0f;  // row 0
  float last = 0.0f;                            // this lane's right-most value, last row done
  float shp = 0.0f;                             // left neighbour's value one row up

  for (int e = tid; e < W * SH; e += S::THREADS) (&sm.ring[0][0])[e] = 0.0f;
  __syncthreads();

  const int steps = nrows + kWave * W - 1 + (W - 1) * LAG;
  const int nint = (steps + KSTEP - 1) / KSTEP;
  for (int it = 0; it < nint; ++it) {
#pragma unroll 1
    for (int s = 0; s < KSTEP; ++s) {
      const int g = it * KSTEP + s;
      const int i = g - delay + 1;              // row of this lane at this step
      // left neighbour's value on row i: DPP from lane-1, or for lane 0 the
      // segment's left column (wave 0) / the previous wave's ring.
      const int i0 = g - lane0_delay + 1;       // row of lane 0 of this wave
      float inj;
      if (wave == 0) {
        inj = (i0 >= 1 && i0 <= nrows) ? sm.left[i0 - 1] : 0.0f;
      } else {
        inj = sm.ring[wave][i0 & (SH - 1)];
      }
      const float shc = wave_shr1(inj, last);
      if (i >= 1 && i <= nrows) {
        const float qi = sm.q[i - 1];
        float cur[C];
        uint32_t code = 0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const float up = dprev[c];
          const float left = c == 0 ? shc : cur[c - 1];
          const float diag = c == 0 ? shp : dprev[c - 1];
          const float mn = min3(up, left, diag);
          if constexpr (DIRS) {
            const uint32_t dcode = diag == mn ? kDirDiag : (up == mn ? kDirUp : kDirLeft);
            code |= dcode << (2 * c);
          }
          cur[c] = mn + local_cost<KIND>(qi, rv[c]);
        }
        if constexpr (DIRS) sm.dirs[(i - 1) * S::THREADS + pos] = (uint8_t)code;
        if constexpr (RIGHT) {
          if (pos == S::THREADS - 1) right[i - 1] = cur[C - 1];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) dprev[c] = cur[c];
        last = cur[C - 1];
      }
      shp = shc;
      if (wave + 1 < W && lane == kWave - 1) {
        const int i63 = g - lane63_delay + 1;
        sm.ring[wave + 1][i63 & (SH - 1)] = last;
      }
    }
    __syncthreads();
  }
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

template <int W, int KIND>
__global__ __launch_bounds__(kWave * W) void sdtw_bwd_kernel(const BwdParams p) {
  using S = BwdShape<W>;
  __shared__ BwdSmem<W> sm;
  __shared__ unsigned long long s_off;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = wave_uniform(tid / kWave);
  const int b = blockIdx.x;
  const int n = wave_uniform(p.lens[b]);
  const int m = p.ref_len;

  int64_t qoff;
  if (p.offsets != nullptr) {
    qoff = p.offsets[b];
  } else {
    if (wave == 0) s_off = 0;
    __syncthreads();
    unsigned long long acc = 0;
    for (int k = tid; k < b; k += S::THREADS) acc += (unsigned long long)p.lens[k];
    atomicAdd(&s_off, acc);
    __syncthreads();
    const unsigned long long v = s_off;
    qoff = (int64_t)(((unsigned long long)(unsigned)wave_uniform((int)(v >> 32)) << 32) |
                     (unsigned)wave_uniform((int)(v & 0xffffffffu)));
  }
  const float* __restrict__ q = p.queries + qoff;
  for (int k = tid; k < n; k += S::THREADS) sm.q[k] = q[k];

  const float gcost = p.grad_cost[b];
  const int K = p.ckpt_every;
  float* __restrict__ gq = p.grad_q + qoff;
  float* __restrict__ part = p.ref_part + (int64_t)b * p.part_stride;
  float* __restrict__ colbuf = p.colbuf + qoff * p.seg_per_block;

  // walker state (uniform; held by wave 0, broadcast through LDS)
  int pi = n;                                   // current row, 1-based
  int pj = wave_uniform((int)p.end_pos[b]);     // current column, 0-based
  float acc_q = 0.0f, acc_r = 0.0f;             // running sums (wave 0)
  int done = 0;
  __syncthreads();

  for (int blk = pj / K; blk >= 0 && !done; --blk) {
    const int bc0 = blk * K;                    // first column of the block
    const int nrows = pi;
    const int seg_last = (pj - bc0) / S::S;     // segment holding the path

    // left boundary of the block: checkpoint blk (column bc0 - 1), or +inf
    auto load_block_left = [&]() {
      if (blk == 0) {
        for (int k = tid; k < nrows; k += S::THREADS) sm.left[k] = inf_f32();
      } else {
        const float* ck = p.ckpt + qoff * p.n_ckpt + (int64_t)(blk - 1) * n;
        for (int k = tid; k < nrows; k += S::THREADS) sm.left[k] = ck[k];
      }
    };
    auto load_seg_ref = [&](int c0) {
      for (int k = tid; k < S::S; k += S::THREADS) {
        const int j = c0 + k;
        sm.rseg[k] = (j < m && j < bc0 + K) ? p.reference[j] : 0.0f;
      }
    };

    // phase 1: right columns of the full segments left of the path's segment
    load_block_left();
    for (int sg = 0; sg < seg_last; ++sg) {
      load_seg_ref(bc0 + sg * S::S);
      __syncthreads();
      float* right = colbuf + (int64_t)sg * n;
      seg_dp<W, KIND, false, true>(sm, nrows, right);
      // next segment's left column = this one's right column
      __syncthreads();
      for (int k = tid; k < nrows; k += S::THREADS) sm.left[k] = right[k];
      __syncthreads();
    }

    // phase 2: segments right to left, directions + walk
    for (int sg = seg_last; sg >= 0 && !done; --sg) {
      const int c0 = bc0 + sg * S::S;
      if (sg == 0) {
        load_block_left();
      } else {
        const float* right = colbuf + (int64_t)(sg - 1) * n;
        for (int k = tid; k < pi; k += S::THREADS) sm.left[k] = right[k];
      }
      load_seg_ref(c0);
      __syncthreads();
      seg_dp<W, KIND, true, false>(sm, pi, nullptr);
      __syncthreads();

      if (wave == 0) {
        // every lane of wave 0 walks the same path (uniform values); lane 0
        // stores
        int i = pi, j = pj;
        for (;;) {
          const float qv = sm.q[i - 1];
          const float rv = sm.rseg[j - c0];
          const float term = gcost * dcost_dq<KIND>(qv, rv);
          acc_q = acc_q + term;
          acc_r = acc_r + (-term);
          if (i == 1) {
            if (lane == 0) {
              gq[0] = acc_q;
              part[j] = acc_r;
              p.path_lo[b] = j;
            }
            done = 1;
            break;
          }
          const int col = j - c0;
          const int byte = sm.dirs[(i - 1) * S::THREADS + (col >> 2)];
          const int code = wave_uniform((byte >> (2 * (col & 3))) & 3);
          if (code != kDirLeft) {               // diagonal or up: leave row i
            if (lane == 0) gq[i - 1] = acc_q;
            acc_q = 0.0f;
            i -= 1;
          }
          if (code != kDirUp) {                 // diagonal or left: leave column j
            if (lane == 0) part[j] = acc_r;
            acc_r = 0.0f;
            j -= 1;
          }
          if (j < c0) break;
        }
        if (lane == 0) {
          sm.state[0] = i;
          sm.state[1] = j;
          sm.state[2] = done;
        }
      }
      __syncthreads();
      pi = wave_uniform(sm.state[0]);
      pj = wave_uniform(sm.state[1]);
      done = wave_uniform(sm.state[2]);
      __syncthreads();
    }
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
