// sdtw_fwd.hpp -- forward sDTW DP fill for gfx950 (wave64, FP32 VALU).
//
// Work mapping (a transposition of the paper's Section 5.2 design, where each
// thread owned a segment of the reference and walked the query rows):
//
//   * one team of W wavefronts per query; lane l of wave w owns R consecutive
//     query rows and keeps their query values and their DP values for the
//     current column in registers;
//   * the reference is streamed in tiles of T columns: at global step g a lane
//     whose team position is L = 64*w + l computes the R x T block of tile
//     tau = g - L - w*LAG;
//   * the DP values of a lane's bottom row for the T columns of a tile feed the
//     next lane one step later through a DPP wave_shr:1 move (the paper's
//     lane shuffle, Section 5.2);
//   * lane 63 of wave w hands its bottom row to lane 0 of wave w+1 through an
//     LDS ring (the paper's shared-memory handoff between consecutive
//     wavefronts); the workgroup synchronises once every KSTEP steps and each
//     wave lags the previous one by an extra LAG = KSTEP-1 steps so that every
//     handoff crosses exactly one barrier;
//   * reference tiles are staged from HBM into an LDS ring by the whole team,
//     one interval ahead;
//   * queries longer than 64*R*W rows are processed in passes; the last row of
//     a pass is written to a global row buffer that seeds the next pass.
//
// The last DP row (row N) is written to the same global row buffer; the
// workgroup then reduces it to its minimum and first minimiser, giving cost
// and end position (paper: Section 2, walk-back start
// "the minimum valued tile in the last row"; Section 5.2 minimum reduction).
//
// Lanes that are still before their first tile (tau < 0) hold +inf in every
// register and only ever see +inf from their neighbours, so they stay +inf
// and need no masking; columns past the end of the reference read zeros and
// produce values nobody reads.
#pragma once

#include "sdtw_argmin.hpp"
#include "sdtw_common.hpp"

namespace sdtw {

struct FwdParams {
  const float* queries;     // packed
  const int32_t* lens;      // [batch]
  const int64_t* offsets;   // [batch + 1] exclusive prefix sum of lens
  const float* reference;   // [ref_len]
  float* rowbuf;            // [slots][row_stride]
  float* cost;              // [batch]   (written by the argmin kernel)
  int64_t* end_pos;         // [batch]
  float* ckpt;              // checkpoint columns, or nullptr
  const int32_t* order;     // persistent form: queries in processing order
  int32_t* queue;           // persistent form: work counter, else nullptr
  int64_t row_stride;       // floats per row-buffer slot (>= ceil(M/T)*T)
  int32_t batch;
  int32_t ref_len;
  int32_t ckpt_every;       // multiple of T when ckpt != nullptr
  int32_t n_ckpt;           // ceil(ref_len / ckpt_every) - 1
};

constexpr int kStepsPerBarrier = 8;

template <int R, int T, int W>
struct FwdShape {
  static constexpr int KSTEP = kStepsPerBarrier;
  static constexpr int LAG = KSTEP - 1;
  static constexpr int SH = 2 * KSTEP;                        // handoff ring, tiles
  static constexpr int SPAN = kWave * W + (W - 1) * LAG + 2 * KSTEP + 2;
  static constexpr int SR = pow2_ceil<SPAN>();                // reference ring, tiles
  static constexpr int THREADS = kWave * W;
  static constexpr int ROWS = kWave * R * W;                  // rows per pass
  static constexpr int CHUNK = KSTEP * T;                     // floats staged per interval
  static constexpr int LDS_FLOATS = SR * T + W * SH * T;
};

// Stage the reference tiles [tile0, tile0 + KSTEP) and the wave-0 top
// boundary (zeros on the first pass, the previous pass's last row after it)
// from global memory into registers.
template <int R, int T, int W>
struct Stager {
  using S = FwdShape<R, T, W>;
  static constexpr int PER = (S::CHUNK + S::THREADS - 1) / S::THREADS;
  float ref[PER];
  float top[PER];

  __device__ __forceinline__ void load(const float* __restrict__ reference, int ref_len,
                                       const float* __restrict__ prev_row, int row_len,
                                       int tile0, int tid) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * S::THREADS;
      const int j = tile0 * T + e;
      float rv = 0.0f, tv = 0.0f;
      if (e < S::CHUNK) {
        if (j < ref_len) rv = reference[j];
        if (prev_row != nullptr && j < row_len) tv = prev_row[j];
      }
      ref[u] = rv;
      top[u] = tv;
    }
  }

  __device__ __forceinline__ void commit(float* s_ref, float* s_hand0, int tile0, int tid) const {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * S::THREADS;
      if (e < S::CHUNK) {
        const int j = tile0 * T + e;
        s_ref[j & (S::SR * T - 1)] = ref[u];
        s_hand0[j & (S::SH * T - 1)] = top[u];
      }
    }
  }
};

// Wavefront index as a value the compiler knows is uniform within a wave, so
// branches on it are scalar branches.
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

__device__ __forceinline__ int64_t uniform_i64(unsigned long long v) {
  const unsigned int hi = (unsigned int)__builtin_amdgcn_readfirstlane((int)(v >> 32));
  const unsigned int lo = (unsigned int)__builtin_amdgcn_readfirstlane((int)(v & 0xffffffffu));
  return (int64_t)(((unsigned long long)hi << 32) | lo);
}

// Process every pass of query b with the team of W waves of this workgroup.
// `row` is this query's row-buffer slot.
template <int R, int T, int W, int KIND, bool CKPT>
__device__ __forceinline__ void fwd_query(const FwdParams& p, int b, int64_t qoff,
                                          float* __restrict__ row, float* s_ref, float* s_hand) {
  using S = FwdShape<R, T, W>;
  constexpr int KSTEP = S::KSTEP, LAG = S::LAG, SH = S::SH, SR = S::SR;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = wave_id();
  const int pos = wave * kWave + lane;                 // lane position in the team

  const int n = __builtin_amdgcn_readfirstlane(p.lens[b]);   // uniform: loop bounds below
  const float* __restrict__ q = p.queries + qoff;
  const int m = p.ref_len;
  const int ntiles = (m + T - 1) / T;
  const int row_len = ntiles * T;
  const int npass = (n + S::ROWS - 1) / S::ROWS;
  const int steps = ntiles + kWave * W - 1 + (W - 1) * LAG;
  const int nint = (steps + KSTEP - 1) / KSTEP;

  for (int pass = 0; pass < npass; ++pass) {
    const int prow0 = pass * S::ROWS;                  // first row of this pass
    const int row0 = prow0 + pos * R;                  // first row of this lane
    float qv[R], dl[R], bot[T];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      qv[k] = (row0 + k < n) ? q[row0 + k] : 0.0f;
      dl[k] = inf_f32();
    }
#pragma unroll
    for (int t = 0; t < T; ++t) bot[t] = inf_f32();
    float corner = inf_f32();

    // Row written to the row buffer by this pass: the pass's last row, or
    // row N on the final pass.
    const bool last_pass = pass == npass - 1;
    const int out_row = last_pass ? (n - 1 - prow0) : (S::ROWS - 1);
    const int out_pos = out_row / R;
    const int out_k = out_row - out_pos * R;
    const int out_wave = out_pos / kWave;
    const int out_lane = out_pos - out_wave * kWave;
    const int out_delay = out_pos + out_wave * LAG;    // out lane's tile = g - out_delay
    const int my_delay = pos + wave * LAG;
    const int lane0_delay = wave * (kWave + LAG);      // lane 0 of this wave
    const int lane63_delay = lane0_delay + kWave - 1;
    const int tiles_per_ckpt = CKPT ? p.ckpt_every / T : 1;
    int ck_cnt = tiles_per_ckpt + my_delay;            // steps until tau = tiles_per_ckpt-1
    int ck_idx = 0;

    // +inf handoff rings (a wave before its first tile must see +inf), then
    // the first interval of reference and top boundary.
    for (int e = tid; e < W * SH * T; e += S::THREADS) s_hand[e] = inf_f32();
    __syncthreads();
    {
      Stager<R, T, W> st;
      st.load(p.reference, m, pass > 0 ? row : nullptr, row_len, 0, tid);
      st.commit(s_ref, s_hand, 0, tid);
    }
    __syncthreads();

    for (int it = 0; it < nint; ++it) {
      Stager<R, T, W> st;
      st.load(p.reference, m, pass > 0 ? row : nullptr, row_len, (it + 1) * KSTEP, tid);

#pragma unroll 1
      for (int s = 0; s < KSTEP; ++s) {
        const int g = it * KSTEP + s;
        const int tau = g - my_delay;
        // top boundary of this lane's block: the previous lane's bottom row
        // (DPP), or for lane 0 the handoff ring of this wave.
        const int tau0 = g - lane0_delay;
        const float* hin = s_hand + wave * SH * T + (tau0 & (SH - 1)) * T;
        const float* rin = s_ref + (tau & (SR - 1)) * T;
        float top[T], rv[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
          top[t] = wave_shr1(hin[t], bot[t]);
          rv[t] = rin[t];
        }

        const int tau_out = g - out_delay;
        const bool do_out = wave == out_wave && tau_out >= 0 && tau_out < ntiles;

        // R x T block, row by row.
        float up[T];
#pragma unroll
        for (int t = 0; t < T; ++t) up[t] = top[t];
        float upleft = corner;                          // D(row-1, first col - 1)
        corner = top[T - 1];
#pragma unroll
        for (int k = 0; k < R; ++k) {
          float left = dl[k];
          float diag = upleft;
          float cur[T];
#pragma unroll
          for (int t = 0; t < T; ++t) {
            const float c = local_cost<KIND>(qv[k], rv[t]);
            const float mn = min3(up[t], left, diag);
            cur[t] = mn + c;
            diag = up[t];
            left = cur[t];
          }
          upleft = dl[k];
          dl[k] = cur[T - 1];
          if (do_out && k == out_k) {
            if (lane == out_lane) {
              float* dst = row + tau_out * T;
#pragma unroll
              for (int t = 0; t < T; ++t) dst[t] = cur[t];
            }
          }
#pragma unroll
          for (int t = 0; t < T; ++t) up[t] = cur[t];
        }
#pragma unroll
        for (int t = 0; t < T; ++t) bot[t] = up[t];

        // lane 63 hands its bottom row to the next wave
        if (wave + 1 < W && lane == kWave - 1) {
          const int tau63 = g - lane63_delay;
          float* hout = s_hand + (wave + 1) * SH * T + (tau63 & (SH - 1)) * T;
#pragma unroll
          for (int t = 0; t < T; ++t) hout[t] = bot[t];
        }

        if constexpr (CKPT) {
          // Checkpoint column kc*ckpt_every - 1 is the last column of a tile
          // (ckpt_every is a multiple of T); a per-lane countdown finds it.
          if (--ck_cnt == 0) {
            ck_cnt = tiles_per_ckpt;
            if (ck_idx < p.n_ckpt) {
              float* dst = p.ckpt + qoff * p.n_ckpt + (int64_t)ck_idx * n + row0;
#pragma unroll
              for (int k = 0; k < R; ++k)
                if (row0 + k < n) dst[k] = dl[k];
            }
            ++ck_idx;
          }
        }
      }
      st.commit(s_ref, s_hand, (it + 1) * KSTEP, tid);
      __syncthreads();
    }
  }
}

// Offset of query b in the packed batch: read from the offset table when the
// host asked for one (large batches), else summed by the workgroup.  No
// thread-dependent branch (see block_argmin).
__device__ __forceinline__ int64_t query_offset(const FwdParams& p, int b) {
  if (p.offsets != nullptr) return p.offsets[b];
  __shared__ unsigned long long s_off;
  if (wave_id() == 0) s_off = 0;
  __syncthreads();
  unsigned long long acc = 0;
  for (int k = threadIdx.x; k < b; k += blockDim.x) acc += (unsigned long long)p.lens[k];
  atomicAdd(&s_off, acc);
  __syncthreads();
  const int64_t off = uniform_i64(s_off);
  __syncthreads();
  return off;
}

// Reduce this query's last DP row (in its row-buffer slot) to cost and end
// position.  The row was written by one lane of this workgroup; the barrier
// makes it visible to every thread.  Wave 0 stores the result (all its
// lanes store the same value).
__device__ __forceinline__ void finish_query(const FwdParams& p, int b, const float* row) {
  __syncthreads();
  const ValIdx x = block_argmin(row, p.ref_len);
  if (wave_id() == 0) {
    p.cost[b] = x.v;
    p.end_pos[b] = x.i;
  }
}

// One workgroup per query.
template <int R, int T, int W, int KIND, bool CKPT>
__global__ __launch_bounds__(kWave * W) void sdtw_fwd_kernel(const FwdParams p) {
  using S = FwdShape<R, T, W>;
  __shared__ __attribute__((aligned(16))) float s_mem[S::LDS_FLOATS];
  const int b = blockIdx.x;
  float* row = p.rowbuf + (int64_t)b * p.row_stride;
  fwd_query<R, T, W, KIND, CKPT>(p, b, query_offset(p, b), row, s_mem, s_mem + S::SR * T);
  finish_query(p, b, row);
}

// Persistent form: a fixed grid pops queries (in the given order, longest
// first) from a device counter; each workgroup owns one row-buffer slot and
// reduces each finished query's last row in place.  Every workgroup leaves
// the loop once the counter passes the batch size.
template <int R, int T, int W, int KIND, bool CKPT>
__global__ __launch_bounds__(kWave * W) void sdtw_fwd_persistent_kernel(const FwdParams p) {
  using S = FwdShape<R, T, W>;
  __shared__ __attribute__((aligned(16))) float s_mem[S::LDS_FLOATS];
  __shared__ int s_item;
  float* row = p.rowbuf + (int64_t)blockIdx.x * p.row_stride;
  // Wave 0 pops the next item: every lane takes part in the atomic (lane 0
  // adds 1, the others 0) so there is no lane-dependent branch; the value is
  // broadcast through LDS.  The item is made wave-uniform with
  // readfirstlane, so the loop, which holds barriers, has a uniform exit.
  const int lane = threadIdx.x & (kWave - 1);
  for (;;) {
    if (wave_id() == 0) {
      const int old = atomicAdd(p.queue, lane == 0 ? 1 : 0);
      s_item = __builtin_amdgcn_readfirstlane(old);
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= p.batch) break;
    const int b = __builtin_amdgcn_readfirstlane(p.order[item]);
    fwd_query<R, T, W, KIND, CKPT>(p, b, query_offset(p, b), row, s_mem, s_mem + S::SR * T);
    finish_query(p, b, row);
  }
}

}  // namespace sdtw
