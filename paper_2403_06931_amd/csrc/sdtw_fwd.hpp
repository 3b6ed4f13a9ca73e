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
//     next lane (the paper's lane shuffle, Section 5.2), either through a
//     per-lane LDS slot or by a DPP wave_shr:1 lane shift (chosen per tile
//     variant).  Lanes lag their neighbour by one step: the value written at
//     the end of step g is read inside step g+1, its LDS latency hidden
//     behind the step's subtractions and products, which do not depend on
//     it.  (On gfx950 DPP moves keep the SIMD from dual-issuing; the LDS form
//     is faster for the large-R tiles, the DPP form for 2-row tiles.)
//   * lane 63 of wave w hands its bottom row to lane 0 of wave w+1 through an
//     LDS ring (the paper's shared-memory handoff between consecutive
//     wavefronts); lane 0 reads it with the same load that reads the other
//     lanes' slots.  The workgroup synchronises once every KSTEP steps and
//     each wave lags the previous one by an extra LAG = KSTEP steps so that
//     every handoff crosses a barrier;
//   * reference tiles are staged from HBM into an LDS ring by the whole team,
//     two barrier intervals ahead;
//   * queries longer than 64*R*W rows are processed in passes; the last row of
//     a pass is written to a global row buffer that seeds the next pass.
//
// The lane holding the stored row writes its values for the step's tile to a
// small LDS buffer.  After each barrier interval its wavefront copies them to
// the row buffer (a pass's last row) or, for row N, folds them into a
// per-lane running (minimum, first minimiser); at the end one wave reduction
// gives cost and end position (Section 2 starts the walk-back from the minimum of the last row;
// Section 5.2 reduces that row to its minimum).  Row N never goes to HBM.
//
// Lanes that are still before their first tile (tau < 0) hold +inf in every
// register and only ever see +inf from their neighbours; the reference slots
// they read are zero-filled at the start of each pass (or hold an earlier
// tile), so their cells are +inf + a finite cost = +inf and need no masking.
// Columns past the end of the reference read zeros and produce values nobody
// reads.
#pragma once

#include "sdtw_argmin.hpp"
#include "sdtw_common.hpp"
#include "sdtw_value.hpp"

namespace sdtw {

struct FwdParams {
  const float* queries;     // packed
  const int32_t* lens;      // [batch]
  const int64_t* offsets;   // [batch + 1] exclusive prefix sum of lens
  const int32_t* ranks;     // [batch] row-buffer slot of each query, with offsets
  const float* reference;   // [ref_len]
  float* rowbuf;            // [slots][row_stride]: one slot per query that needs
                            // several row passes (plain launch) or per workgroup
                            // (persistent launch)
  float* cost;              // [batch]   (written by the argmin kernel)
  int64_t* end_pos;         // [batch]
  float* ckpt;              // checkpoint columns, or nullptr
  float* rowck;             // row checkpoints (with ckpt), or nullptr
  const int32_t* order;     // persistent form: queries in processing order
  int32_t* queue;           // persistent form: work counter, else nullptr
  int64_t row_stride;       // floats per row-buffer slot (>= ceil(M/T)*T)
  int32_t batch;
  int32_t ref_len;
  int32_t ckpt_every;       // multiple of T when ckpt != nullptr
  int32_t n_ckpt;           // ceil(ref_len / ckpt_every) - 1
  float prune_tau;          // pruning threshold of the kPruned cost kind
};

constexpr int kStepsPerBarrier = 8;

template <int R, int T, int W, int KS, int XL>
struct FwdShape {
  static_assert(KS % 2 == 0, "the step loop is unrolled by two");
  static constexpr int KSTEP = KS;
  // lane -> lane exchange: XL = 1 through LDS slots, XL = 0 through a DPP
  // wave_shr:1 move; either way lane l+1 lags lane l by one step (a slot is
  // read inside the step that uses it, after the neighbour's write at the
  // end of the previous step)
  static constexpr int LL = 1;
  // Extra lag of wave w+1 behind wave w.  Data a wave hands over at step p is
  // used at step p + KS + 1 (read inside that step with XL, by the prefetch
  // one step earlier without), always in a later barrier interval.
  static constexpr int LAG = KS;
  static constexpr int SH = 4 * KS;                           // handoff rings, tiles
  // reference tiles in flight: the oldest lane's tile up to the tiles staged
  // two intervals ahead
  static constexpr int SPAN = LL * kWave * W + (W - 1) * LAG + 3 * KS + 2;
  static constexpr int SR = pow2_ceil<SPAN>();                // reference ring, tiles
  static constexpr int THREADS = kWave * W;
  static constexpr int ROWS = kWave * R * W;                  // rows per pass
  static constexpr int CHUNK = KS * T;                        // floats staged per interval
  static constexpr int SLOTS = XL ? W * kWave * T : 0;        // lane -> lane slots
  static constexpr int OUTBUF = KS * T;                       // row N over one interval
  // R = 8: the row checkpoint in the middle of each wavefront, one ring per
  // wavefront like the handoff rings
  // (checkpointing kernels only, after the other buffers)
  static constexpr int MIDRING = R * kWave > kRowCkpt ? W * SH * T : 0;
  static constexpr int LDS_FLOATS = SR * T + W * SH * T + SLOTS + OUTBUF;
  template <bool CKPT>
  static constexpr int lds_floats() { return LDS_FLOATS + (CKPT ? MIDRING : 0); }
};

// Stage the reference tiles [tile0, tile0 + KS) and the wave-0 top boundary
// (zeros on the first pass, the previous pass's last row after it) from
// global memory into registers; commit them to the LDS rings later.
template <int R, int T, int W, int KS, int XL, typename V = float>
struct Stager {
  using S = FwdShape<R, T, W, KS, XL>;
  static constexpr int PER = (S::CHUNK + S::THREADS - 1) / S::THREADS;
  using In = typename Val<V>::In;
  In ref[PER];
  V top[PER];

  __device__ __forceinline__ void load(const float* __restrict__ reference_in, int ref_len,
                                       const V* __restrict__ prev_row, int row_len,
                                       int tile0, int tid) {
    const In* __restrict__ reference = reinterpret_cast<const In*>(reference_in);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * S::THREADS;
      const int j = tile0 * T + e;
      In rv = In(0);
      V tv = Val<V>::zero();
      if (e < S::CHUNK) {
        if (j < ref_len) rv = reference[j];
        if (prev_row != nullptr && j < row_len) tv = prev_row[j];
      }
      ref[u] = rv;
      top[u] = tv;
    }
  }

  __device__ __forceinline__ void commit(V* s_ref, V* s_hand0, int tile0, int tid) const {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * S::THREADS;
      if (e < S::CHUNK) {
        const int j = tile0 * T + e;
        s_ref[j & (S::SR * T - 1)] = Val<V>::ref(ref[u]);
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

// Thread and wavefront index within the team of W wavefronts that works on
// one query (a workgroup of the persistent form holds several one-wavefront
// teams), and the team's barrier: with W = 1 every LDS exchange stays inside
// one wavefront, whose LDS operations complete in issue order, so a fence
// that keeps the compiler from moving them across it is enough.
template <int W>
__device__ __forceinline__ int team_tid() {
  return (int)(threadIdx.x % (kWave * W));
}

template <int W>
__device__ __forceinline__ int team_wave() {
  return __builtin_amdgcn_readfirstlane((int)((threadIdx.x / kWave) % W));
}

template <int W>
__device__ __forceinline__ void team_sync() {
  if constexpr (W == 1) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One-wavefront teams per workgroup of the persistent form.
__host__ __device__ constexpr int persistent_teams(int W) { return W == 1 ? 4 : 1; }

__device__ __forceinline__ int64_t uniform_i64(unsigned long long v) {
  const unsigned int hi = (unsigned int)__builtin_amdgcn_readfirstlane((int)(v >> 32));
  const unsigned int lo = (unsigned int)__builtin_amdgcn_readfirstlane((int)(v & 0xffffffffu));
  return (int64_t)(((unsigned long long)hi << 32) | lo);
}

// Per-lane DP state of one pass (V: one binary32 query per lane row, or two
// binary16 queries packed in halves).
template <int R, int T, typename V = float>
struct LaneState {
  V qv[R];         // query values of the lane's rows
  V dl[R];         // DP values of the lane's rows at the last column done
  V bot[T];        // the lane's bottom row over the last tile (feeds lane + 1)
  V corner;        // top boundary at the column before the current tile
  int ck_h;        // step at which the lane reaches its next checkpoint column
  int ck_k;        // index of that checkpoint (0-based)
  float ckv[R];    // the lane's rows at the last checkpoint column reached
  ValIdx am[Val<V>::N];   // running (minimum, first minimiser) of row N, per query
  float tau;       // pruning threshold (kPruned), held in a vector register
};

// Uniform (per wavefront) geometry of one pass.
struct PassGeom {
  int wave, lane, row0, n, ntiles, nint;
  int my_delay, lane0_delay, lane63_delay;   // tile = step - delay
  int out_delay, out_lane;                   // lane holding the row to store
  int tiles_per_ckpt;
  bool ck_each_step;                         // store checkpoints every step
  bool final_pass;                           // the stored row is row N
  bool idle;                                 // every row of this wave is past row N
  float* rowck;                              // row checkpoint this wave copies, or nullptr
  float* rowck_mid;                          // row checkpoint inside this wave, or nullptr
  int64_t qoff;
  float* row;                                // row-buffer slot of the query
  float* s_out;                              // LDS: row N over one interval
  float* s_mid;                              // LDS: mid-wavefront checkpoint rings
};

// Store the lane's rows at checkpoint column ck_k from `v` and move on to
// the next checkpoint.
template <int R, int T>
__device__ __forceinline__ void ckpt_store(const FwdParams& p, LaneState<R, T>& L,
                                           const PassGeom& G, const float (&v)[R]) {
  if (L.ck_k < p.n_ckpt) {
    float* dst = p.ckpt + G.qoff * p.n_ckpt + (int64_t)L.ck_k * G.n + G.row0;
#pragma unroll
    for (int k = 0; k < R; ++k)
      if (G.row0 + k < G.n) __builtin_nontemporal_store(v[k], &dst[k]);
  }
  L.ck_h += G.tiles_per_ckpt;
  ++L.ck_k;
}

// End of barrier interval `it`: store the checkpoint column captured in it,
// if the lane reached one (checkpoints are at least one interval apart here,
// so a lane reaches at most one per interval).
template <int R, int T, int KS>
__device__ __forceinline__ void ckpt_flush(const FwdParams& p, LaneState<R, T>& L,
                                           const PassGeom& G, int it) {
  if (L.ck_h < (it + 1) * KS) ckpt_store(p, L, G, L.ckv);
}

// Row checkpoints D(kRowCkpt*k, 1..M) for every multiple of kRowCkpt below
// N.  With checkpoints every pass holds R rows per lane.  For R = 2 and 4,
// kRowCkpt is a multiple of a wavefront's 64*R rows, so such a row is the
// bottom row of a wavefront, or else the last row of a pass, which the next
// pass stages into wavefront 0's ring: the wavefront whose ring carries it
// copies the tiles it read in barrier interval `it` to global memory at the
// interval's end (a tile stays in the ring for two more intervals after its
// read).  For R = 8 a wavefront holds 2*kRowCkpt rows, and the one in its
// middle is the bottom row of lane kRowCkpt/R - 1, which goes through a ring
// of its own (rowck_mid_put, rowck_mid_copy).  Checkpoint stores are non-temporal: the
// backward reads a fraction of them, later, and they should not leave the
// caches full of dirty lines.
template <int T, int KS, int SH>
__device__ __forceinline__ void rowck_copy(const FwdParams& p, const PassGeom& G,
                                           const float* s_hand, int it) {
  const float* ring = s_hand + G.wave * SH * T;
  const int tau0 = it * KS - G.lane0_delay;
#pragma unroll
  for (int e0 = 0; e0 < KS * T; e0 += kWave) {
    const int e = e0 + G.lane;
    if (e < KS * T) {
      const int tau = tau0 + e / T;
      const int col = tau * T + (e & (T - 1));
      if (tau >= 0 && col < p.ref_len) {
        const float v = ring[(tau & (SH - 1)) * T + (e & (T - 1))];
        __builtin_nontemporal_store(v, &G.rowck[col]);
      }
    }
  }
}

// Checkpoint handling inside the step loop: none, capture the checkpoint
// column with selects (stored at the interval's end), or store it in the
// step that reaches it (checkpoints closer than one barrier interval).
enum CkptMode { kCkNone = 0, kCkSelect = 1, kCkEachStep = 2 };

// The row checkpoint inside a wavefront of R = 8 rows per lane: lane
// kRowCkpt/R - 1 writes its bottom row over the tile of step g into its
// wavefront's ring, and at the end of each barrier interval the wavefront
// copies the tiles of that interval to global memory (rowck_mid_copy), as
// for the rows handed over at wavefront boundaries.
template <int R, int T, int SH>
__device__ __forceinline__ void rowck_mid_put(const PassGeom& G, const float (&bot)[T], int g) {
  static_assert(R * kWave == 2 * kRowCkpt, "one row checkpoint inside a wavefront");
  if (G.rowck_mid != nullptr && G.lane == kRowCkpt / R - 1) {
    float* dst = G.s_mid + (G.wave * SH + ((g - G.my_delay) & (SH - 1))) * T;
#pragma unroll
    for (int t = 0; t < T; ++t) dst[t] = bot[t];
  }
}

template <int R, int T, int KS, int SH>
__device__ __forceinline__ void rowck_mid_copy(const FwdParams& p, const PassGeom& G, int it) {
  const float* ring = G.s_mid + G.wave * SH * T;
  const int tau0 = it * KS - (G.lane0_delay + kRowCkpt / R - 1);
#pragma unroll
  for (int e0 = 0; e0 < KS * T; e0 += kWave) {
    const int e = e0 + G.lane;
    if (e < KS * T) {
      const int tau = tau0 + e / T;
      const int col = tau * T + (e & (T - 1));
      if (tau >= 0 && tau < G.ntiles && col < p.ref_len)
        __builtin_nontemporal_store(ring[(tau & (SH - 1)) * T + (e & (T - 1))],
                                    &G.rowck_mid[col]);
    }
  }
}

// One step: the R x T block of this lane's current tile.  OUTK >= 0 marks
// the wavefront holding the row to store and that row's register index.
// `top` is the block's top boundary: the previous lane's bottom row over this
// tile (for lane 0, the previous wave's, or the top boundary of the pass).
template <int R, int T, int W, int KS, int XL, int KIND, int CKM, int OUTK, typename V>
__device__ __forceinline__ void fwd_step(const FwdParams& p, LaneState<R, T, V>& L,
                                         const PassGeom& G, const V (&rv)[T],
                                         const V (&top)[T], int g, V* s_hand, V* s_slot) {
  using S = FwdShape<R, T, W, KS, XL>;
  V up[T];
  if constexpr (XL) {
    // lane l-1's slot, written at the end of step g-1 (lane 0: this wave's
    // handoff ring); the read's latency is covered by the block's
    // subtractions and products, which do not depend on it
    const V* hin = s_hand + G.wave * S::SH * T + ((g - G.lane0_delay) & (S::SH - 1)) * T;
    const V* tin = G.lane != 0 ? s_slot + (G.wave * kWave + G.lane - 1) * T : hin;
#pragma unroll
    for (int t = 0; t < T; ++t) up[t] = tin[t];
  } else {
#pragma unroll
    for (int t = 0; t < T; ++t) up[t] = Val<V>::shr1(top[t], L.bot[t]);
  }
  V upleft = L.corner;                          // D(row-1, first col - 1)
  L.corner = up[T - 1];
  const int tau_out = g - G.out_delay;
  const bool do_out = OUTK >= 0 && tau_out >= 0 && tau_out < G.ntiles;
  if constexpr (Val<V>::kAntiDiagonal) {
    // Anti-diagonal order (packed binary16): gfx950 needs a wait state
    // between dependent packed instructions; cells (k, t) and (k+1, t-1)
    // are independent, so this order puts independent work between them.
    V D[R][T];
#pragma unroll
    for (int d = 0; d < R + T - 1; ++d) {
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int t = d - k;
        if (t < 0 || t >= T) continue;
        const V u = k == 0 ? up[t] : D[k - 1][t];
        const V lf = t == 0 ? L.dl[k] : D[k][t - 1];
        const V dg = t == 0 ? (k == 0 ? upleft : L.dl[k - 1]) : (k == 0 ? up[t - 1] : D[k - 1][t - 1]);
        D[k][t] = Val<V>::template cell<KIND>(L.qv[k], rv[t], u, lf, dg, L.tau);
      }
    }
    if constexpr (OUTK >= 0) {
      if (do_out && G.lane == G.out_lane) {
        V* dst = reinterpret_cast<V*>(G.s_out) + (g & (KS - 1)) * T;
#pragma unroll
        for (int t = 0; t < T; ++t) dst[t] = D[OUTK][t];
      }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) L.dl[k] = D[k][T - 1];
#pragma unroll
    for (int t = 0; t < T; ++t) up[t] = D[R - 1][t];
  } else {
  // The block row by row (measured faster on gfx950 than anti-diagonal
  // order, which the compiler schedules worse for dual issue).
#pragma unroll
  for (int k = 0; k < R; ++k) {
    V left = L.dl[k];
    V diag = upleft;
    V cur[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      cur[t] = Val<V>::template cell<KIND>(L.qv[k], rv[t], up[t], left, diag, L.tau);
      diag = up[t];
      left = cur[t];
    }
    upleft = L.dl[k];
    L.dl[k] = cur[T - 1];
    if (OUTK == k) {                            // folded once the k loop is unrolled
      if (do_out && G.lane == G.out_lane) {
        // to LDS only: at the interval's end the wave folds it (row N) or
        // copies it to the row buffer (keeping a global store out of the
        // step, whose LDS waits would otherwise cover it)
        V* dst = reinterpret_cast<V*>(G.s_out) + (g & (KS - 1)) * T;
#pragma unroll
        for (int t = 0; t < T; ++t) dst[t] = cur[t];
      }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) up[t] = cur[t];
  }
  }
#pragma unroll
  for (int t = 0; t < T; ++t) L.bot[t] = up[t];

  if constexpr (XL) {
    // the bottom row feeds lane l+1 (its slot is read at the start of the
    // next step, before this lane overwrites it at the end of that step).
    // LDS operations of one wavefront complete in order; the compiler must
    // not move the next step's slot read (another lane's slot, so no alias
    // in one thread's view) above this store.
    V* sout = s_slot + (G.wave * kWave + G.lane) * T;
#pragma unroll
    for (int t = 0; t < T; ++t) sout[t] = L.bot[t];
    asm volatile("" ::: "memory");
  }

  // lane 63 hands its bottom row to the next wave
  if (G.wave + 1 < W && G.lane == kWave - 1) {
    V* hout = s_hand + (G.wave + 1) * S::SH * T + ((g - G.lane63_delay) & (S::SH - 1)) * T;
#pragma unroll
    for (int t = 0; t < T; ++t) hout[t] = L.bot[t];
  }

  // Checkpoint column kc*ckpt_every - 1 is the last column of tile kc*tpc - 1
  // (tpc = tiles per checkpoint; ckpt_every is a multiple of T), which the
  // lane reaches at step my_delay + kc*tpc - 1.
  if constexpr (CKM == kCkEachStep) {
    if (g == L.ck_h) ckpt_store(p, L, G, L.dl);
  } else if constexpr (CKM == kCkSelect) {
    const bool hit = g == L.ck_h;
#pragma unroll
    for (int k = 0; k < R; ++k) L.ckv[k] = hit ? L.dl[k] : L.ckv[k];
  }
  if constexpr (CKM != kCkNone && R * kWave > kRowCkpt)
    rowck_mid_put<R, T, FwdShape<R, T, W, KS, XL>::SH>(G, L.bot, g);
}

// LDS inputs of step g, read one step ahead: this lane's reference tile and,
// without XL, the handoff ring's top boundary (fwd_step shifts the bottom
// rows to the other lanes); with XL, fwd_step reads the top boundary itself.
template <int R, int T, int W, int KS, int XL, typename V>
__device__ __forceinline__ void step_inputs(V (&rv)[T], V (&top)[T], int g, const PassGeom& G,
                                            const V* s_ref, const V* s_hand, const V* s_slot) {
  using S = FwdShape<R, T, W, KS, XL>;
  const V* rin = s_ref + ((g - G.my_delay) & (S::SR - 1)) * T;
  const V* hin = s_hand + G.wave * S::SH * T + ((g - G.lane0_delay) & (S::SH - 1)) * T;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    rv[t] = rin[t];
    if constexpr (!XL) top[t] = hin[t];
  }
}

// Fold the row-N values the out lane wrote during interval `it` (tiles
// it*KS + s - out_delay, s < KS) into this lane's running (minimum, first
// minimiser), one per query of the value.  A lane sees the columns in
// increasing order, so a strict comparison keeps the first minimiser.
template <int T, int KS, typename V>
__device__ __forceinline__ void out_fold(ValIdx (&am)[Val<V>::N], const PassGeom& G, int it,
                                         int ref_len) {
  const V* s_out = reinterpret_cast<const V*>(G.s_out);
  for (int e = G.lane; e < KS * T; e += kWave) {
    const int tau = it * KS + e / T - G.out_delay;
    const int j = tau * T + e % T;
    const V x = s_out[e];
    const bool in = tau >= 0 && tau < G.ntiles && j < ref_len;
#pragma unroll
    for (int h = 0; h < Val<V>::N; ++h) {
      const float v = Val<V>::half(x, h);
      if (in && v < am[h].v) {
        am[h].v = v;
        am[h].i = j;
      }
    }
  }
}

// Copy the stored row's values of interval `it` from LDS to the row buffer
// (a pass's last row, read by the next pass).
template <int T, int KS>
__device__ __forceinline__ void out_copy(const PassGeom& G, int it) {
  // (non-temporal: the next pass reads these values a whole pass later,
  // long after they would have left the caches; cached, they would only
  // displace the reference tiles every workgroup re-reads)
  for (int e = G.lane; e < KS * T; e += kWave) {
    const int tau = it * KS + e / T - G.out_delay;
    if (tau >= 0 && tau < G.ntiles)
      __builtin_nontemporal_store(G.s_out[e], &G.row[tau * T + e % T]);
  }
}

// The KS steps of barrier interval `it`.  The reference tile of step g+1
// (and, without XL, its handoff input) is read while step g computes (two
// register sets, the step loop unrolled by two).
template <int R, int T, int W, int KS, int XL, int KIND, int CKM, int OUTK, typename V>
__device__ __forceinline__ void fwd_steps(const FwdParams& p, LaneState<R, T, V>& L,
                                          const PassGeom& G, int it, V (&rvA)[T], V (&injA)[T],
                                          V (&rvB)[T], V (&injB)[T], const V* s_ref, V* s_hand,
                                          V* s_slot) {
#pragma unroll 1
  for (int s = 0; s < KS; s += 2) {
    const int g = it * KS + s;
    step_inputs<R, T, W, KS, XL>(rvB, injB, g + 1, G, s_ref, s_hand, s_slot);
    fwd_step<R, T, W, KS, XL, KIND, CKM, OUTK, V>(p, L, G, rvA, injA, g, s_hand, s_slot);
    step_inputs<R, T, W, KS, XL>(rvA, injA, g + 2, G, s_ref, s_hand, s_slot);
    fwd_step<R, T, W, KS, XL, KIND, CKM, OUTK, V>(p, L, G, rvB, injB, g + 1, s_hand, s_slot);
  }
}

// All barrier intervals of one pass.
template <int R, int T, int W, int KS, int XL, int KIND, bool CKPT, int OUTK, typename V>
__device__ __forceinline__ void fwd_pass(const FwdParams& p, LaneState<R, T, V>& L,
                                         const PassGeom& G, const V* prev_row, V* s_ref,
                                         V* s_hand, V* s_slot) {
  const int tid = team_tid<W>();
  V rvA[T], injA[T], rvB[T], injB[T];
  step_inputs<R, T, W, KS, XL>(rvA, injA, 0, G, s_ref, s_hand, s_slot);
  for (int it = 0; it < G.nint; ++it) {
    Stager<R, T, W, KS, XL, V> st;
    st.load(p.reference, p.ref_len, prev_row, G.ntiles * T, (it + 2) * KS, tid);
    // A wave whose rows all lie past row N (the last pass of a query that
    // does not fill it) computes nothing: nothing flows upward, so its cells
    // are never read.  It still stages its share of the reference and meets
    // every barrier; its issue slots go to the other waves on its SIMD.
    // (the checkpoint mode is a loop-invariant choice, taken outside the
    // step loop so that the loop holds only the chosen form's instructions)
    if (!G.idle) {
      if constexpr (CKPT) {
        if (G.ck_each_step)
          fwd_steps<R, T, W, KS, XL, KIND, kCkEachStep, OUTK, V>(p, L, G, it, rvA, injA, rvB,
                                                                 injB, s_ref, s_hand, s_slot);
        else
          fwd_steps<R, T, W, KS, XL, KIND, kCkSelect, OUTK, V>(p, L, G, it, rvA, injA, rvB, injB,
                                                               s_ref, s_hand, s_slot);
      } else {
        fwd_steps<R, T, W, KS, XL, KIND, kCkNone, OUTK, V>(p, L, G, it, rvA, injA, rvB, injB,
                                                           s_ref, s_hand, s_slot);
      }
    }
    // The stager's commit waits for its loads with a vmcnt wait, which on
    // gfx950 also covers every store issued before it; the interval's global
    // stores (checkpoints, a pass's last row) therefore come after the
    // commit and complete while the next interval computes.
    st.commit(s_ref, s_hand, (it + 2) * KS, tid);
    if constexpr (CKPT) {
      if (!G.ck_each_step) ckpt_flush<R, T, KS>(p, L, G, it);
      if (G.rowck != nullptr)
        rowck_copy<T, KS, FwdShape<R, T, W, KS, XL>::SH>(p, G, reinterpret_cast<float*>(s_hand),
                                                          it);
      if constexpr (R * kWave > kRowCkpt) {
        if (G.rowck_mid != nullptr)
          rowck_mid_copy<R, T, KS, FwdShape<R, T, W, KS, XL>::SH>(p, G, it);
      }
    }
    if constexpr (OUTK >= 0) {
      if (G.final_pass) {
        out_fold<T, KS, V>(L.am, G, it, p.ref_len);
      } else {
        out_copy<T, KS>(G, it);
      }
    }
    team_sync<W>();
  }
}

// The wavefront holding the stored row runs a copy of the pass with that
// row's register index as a compile-time constant; the others store nothing.
template <int K, int R, int T, int W, int KS, int XL, int KIND, bool CKPT, typename V>
__device__ __forceinline__ void fwd_pass_out(int out_k, const FwdParams& p,
                                             LaneState<R, T, V>& L, const PassGeom& G,
                                             const V* prev_row, V* s_ref, V* s_hand, V* s_slot) {
  if constexpr (K < R) {
    if (out_k == K) {
      fwd_pass<R, T, W, KS, XL, KIND, CKPT, K, V>(p, L, G, prev_row, s_ref, s_hand, s_slot);
    } else {
      fwd_pass_out<K + 1, R, T, W, KS, XL, KIND, CKPT, V>(out_k, p, L, G, prev_row, s_ref,
                                                          s_hand, s_slot);
    }
  }
}

// One pass of query b: rows [prow0, prow0 + 64 RR W) held RR per lane.  The
// tile schedule (delays, rings, barriers) does not depend on RR, so any RR
// computes the same cells bit for bit; RR only decides how many rows a pass
// covers and how they are spread over the lanes.
template <int RR, int T, int W, int KS, int XL, int KIND, bool CKPT, typename V>
__device__ __forceinline__ void fwd_one_pass(const FwdParams& p, int b, PassGeom& G, int pos,
                                             int prow0, int pass_rows, bool last_pass,
                                             const typename Val<V>::In* __restrict__ q,
                                             const typename Val<V>::In* __restrict__ q2,
                                             const V* prev_row, V* s_ref, V* s_hand,
                                             V* s_slot) {
  using S = FwdShape<RR, T, W, KS, XL>;
  using In = typename Val<V>::In;
  const int tid = team_tid<W>();
  G.row0 = prow0 + pos * RR;                           // first row of this lane
  G.idle = prow0 + G.wave * kWave * RR >= G.n;         // uniform: wave and lengths
  // the row above this wave's first row, if it is a row checkpoint
  const int bnd = prow0 + G.wave * kWave * RR;
  G.rowck = CKPT && p.rowck != nullptr && bnd > 0 && bnd % kRowCkpt == 0 && bnd < G.n
                ? p.rowck + (G.qoff / kRowCkpt + bnd / kRowCkpt - 1) * (int64_t)p.ref_len
                : nullptr;
  // (RR = 8: the row kRowCkpt below that one lies inside this wave)
  const int mid = bnd + kRowCkpt;
  G.rowck_mid = CKPT && RR * kWave > kRowCkpt && p.rowck != nullptr && mid % kRowCkpt == 0 &&
                        mid < G.n
                    ? p.rowck + (G.qoff / kRowCkpt + mid / kRowCkpt - 1) * (int64_t)p.ref_len
                    : nullptr;
  LaneState<RR, T, V> L;
#pragma unroll
  for (int k = 0; k < RR; ++k) {
    const bool in = G.row0 + k < G.n;
    if constexpr (Val<V>::N == 1) {
      L.qv[k] = Val<V>::query(in ? q[G.row0 + k] : In(0), In(0));
    } else {
      L.qv[k] = Val<V>::query(in ? q[G.row0 + k] : 0.0f, in ? q2[G.row0 + k] : 0.0f);
    }
    L.dl[k] = Val<V>::inf();
  }
#pragma unroll
  for (int t = 0; t < T; ++t) L.bot[t] = Val<V>::inf();
  L.corner = Val<V>::inf();
  L.ck_h = G.my_delay + G.tiles_per_ckpt - 1;          // reaches checkpoint 0 there
  L.ck_k = 0;
#pragma unroll
  for (int k = 0; k < RR; ++k) L.ckv[k] = 0.0f;
#pragma unroll
  // (+inf, column 0): a row that is +inf throughout (an overflow) folds
  // nothing and reports its first column, the smallest index attaining
  // the minimum; any finite value replaces it
  for (int h = 0; h < Val<V>::N; ++h) L.am[h] = ValIdx{inf_f32(), 0};
  L.tau = 0.0f;
  if constexpr (KIND == kPruned) L.tau = vgpr_copy(p.prune_tau);

  // Row stored by this pass: the pass's last row (to the row buffer), or
  // row N on the final pass (reduced on the fly).
  G.final_pass = last_pass;
  const int out_row = last_pass ? (G.n - 1 - prow0) : (pass_rows - 1);
  const int out_pos = out_row / RR;
  const int out_k = out_row - out_pos * RR;
  const int out_wave = out_pos / kWave;
  G.out_lane = out_pos - out_wave * kWave;
  G.out_delay = S::LL * out_pos + out_wave * S::LAG;  // out lane's tile = step - out_delay

  // +inf handoff rings and lane slots (a lane before its first tile must
  // see +inf), a zeroed reference ring (so that those lanes compute on
  // finite values, never on whatever the LDS held), then the first two
  // intervals of reference and top boundary.
  for (int e = tid; e < W * S::SH * T; e += S::THREADS) s_hand[e] = Val<V>::inf();
  for (int e = tid; e < S::SLOTS; e += S::THREADS) s_slot[e] = Val<V>::inf();
  for (int e = tid; e < S::SR * T; e += S::THREADS) s_ref[e] = Val<V>::zero();
  team_sync<W>();
  {
    Stager<RR, T, W, KS, XL, V> st0, st1;
    st0.load(p.reference, p.ref_len, prev_row, G.ntiles * T, 0, tid);
    st1.load(p.reference, p.ref_len, prev_row, G.ntiles * T, KS, tid);
    st0.commit(s_ref, s_hand, 0, tid);
    st1.commit(s_ref, s_hand, KS, tid);
  }
  team_sync<W>();

  if (G.wave == out_wave) {
    fwd_pass_out<0, RR, T, W, KS, XL, KIND, CKPT, V>(out_k, p, L, G, prev_row, s_ref, s_hand,
                                                     s_slot);
    if (last_pass) {
      // every lane of the wave holds the result and stores it (no
      // lane-dependent branch in a loop that holds barriers)
#pragma unroll
      for (int h = 0; h < Val<V>::N; ++h) {
        if (h == 0 || b + h < p.batch) {
          const ValIdx x = wave_argmin(L.am[h]);
          p.cost[b + h] = x.v;
          p.end_pos[b + h] = x.i;
        }
      }
    }
  } else {
    fwd_pass<RR, T, W, KS, XL, KIND, CKPT, -1, V>(p, L, G, prev_row, s_ref, s_hand, s_slot);
  }
}

// Rows per lane of the shortest tail pass fwd_query may use with R rows per
// lane in its full passes (R itself: no tail form).
template <int R>
constexpr int tail_rows_min() {
  return R >= 8 ? R / 4 : (R >= 4 ? R / 2 : R);
}

// Process every pass of query b (with f16x2 values: queries b and b+1, of
// equal length, or b twice when it is the batch's last) with the team of W
// waves of this workgroup and store cost and end position.  `row` is the
// row-buffer slot (rows carried from one pass to the next, as V words).
// Full passes hold R rows per lane.  With RT < R the last pass, when its
// rows fit, holds R/2 or (if RT allows) R/4 or 3R/4 rows per lane instead,
// the fewest that hold them: fewer padding rows below row N for a query
// that is not a multiple of a pass long, at a somewhat higher cost per cell.
template <int R, int T, int W, int KS, int XL, int KIND, bool CKPT, typename V = float,
          int RT = R>
__device__ __forceinline__ void fwd_query(const FwdParams& p, int b, int64_t qoff,
                                          float* __restrict__ row, float* s_mem) {
  static_assert(!CKPT || Val<V>::N == 1, "checkpoints are binary32 only");
  static_assert(RT == R || RT == R / 2 || RT == R / 4, "tail passes hold R/2 or R/4 rows");
  using S0 = FwdShape<R, T, W, KS, XL>;
  V* s_ref = reinterpret_cast<V*>(s_mem);
  V* s_hand = s_ref + S0::SR * T;
  V* s_slot = s_hand + W * S0::SH * T;
  using S = FwdShape<R, T, W, KS, XL>;
  const int tid = team_tid<W>();
  PassGeom G;
  G.lane = tid & (kWave - 1);
  G.wave = team_wave<W>();
  const int pos = G.wave * kWave + G.lane;             // lane position in the team
  G.n = __builtin_amdgcn_readfirstlane(p.lens[b]);     // uniform: loop bounds below
  G.qoff = qoff;
  G.row = row;
  G.s_out = reinterpret_cast<float*>(s_slot + S0::SLOTS);
  G.s_mid = G.s_out + S0::OUTBUF;
  using In = typename Val<V>::In;
  const In* __restrict__ q = reinterpret_cast<const In*>(p.queries) + qoff;
  // second query of a binary16 pair (the same one at the end of an odd batch)
  const In* __restrict__ q2 = (Val<V>::N > 1 && b + 1 < p.batch) ? q + G.n : q;
  G.ntiles = (p.ref_len + T - 1) / T;
  const int npass = (G.n + S::ROWS - 1) / S::ROWS;
  const int steps = G.ntiles + S::LL * (kWave * W - 1) + (W - 1) * S::LAG;
  G.nint = (steps + KS - 1) / KS;
  G.my_delay = S::LL * pos + G.wave * S::LAG;
  G.lane0_delay = G.wave * (S::LL * kWave + S::LAG);
  G.lane63_delay = G.lane0_delay + S::LL * (kWave - 1);
  G.tiles_per_ckpt = CKPT ? p.ckpt_every / T : 1;
  G.ck_each_step = G.tiles_per_ckpt < KS;

  for (int pass = 0; pass < npass; ++pass) {
    const int prow0 = pass * S::ROWS;                  // first row of this pass
    const bool last_pass = pass == npass - 1;
    const V* prev_row = pass > 0 ? reinterpret_cast<const V*>(row) : nullptr;
    if constexpr (RT < R) {
      const int left = G.n - prow0;                    // rows of this pass, uniform
      if constexpr (RT <= R / 4) {
        if (last_pass && left <= kWave * W * (R / 4)) {
          fwd_one_pass<R / 4, T, W, KS, XL, KIND, CKPT, V>(p, b, G, pos, prow0, left, true, q,
                                                           q2, prev_row, s_ref, s_hand, s_slot);
          continue;
        }
      }
      if (last_pass && left <= kWave * W * (R / 2)) {
        fwd_one_pass<R / 2, T, W, KS, XL, KIND, CKPT, V>(p, b, G, pos, prow0, left, true, q, q2,
                                                         prev_row, s_ref, s_hand, s_slot);
        continue;
      }
      if constexpr (RT <= R / 4) {
        if (last_pass && left <= kWave * W * (3 * R / 4)) {
          fwd_one_pass<3 * R / 4, T, W, KS, XL, KIND, CKPT, V>(p, b, G, pos, prow0, left, true,
                                                               q, q2, prev_row, s_ref, s_hand,
                                                               s_slot);
          continue;
        }
      }
    }
    fwd_one_pass<R, T, W, KS, XL, KIND, CKPT, V>(p, b, G, pos, prow0, S::ROWS, last_pass, q, q2,
                                                 prev_row, s_ref, s_hand, s_slot);
  }
}

// Where query b sits: its offset in the packed batch and, for the plain
// launch, its row-buffer slot (the number of earlier queries longer than
// `rows`, one pass of the tile; a query that fits in one pass never touches
// the row buffer).  Read from the tables the host asked for (large batches),
// else summed by the workgroup.  No thread-dependent branch (a loop of the
// persistent kernel holds barriers).
struct QueryPos {
  int64_t off;
  int32_t slot;
};

__device__ __forceinline__ QueryPos query_pos(const FwdParams& p, int b, int rows) {
  if (p.offsets != nullptr)
    return QueryPos{p.offsets[b], p.ranks != nullptr ? p.ranks[b] : 0};
  __shared__ unsigned long long s_off;
  __shared__ int s_slot;
  if (wave_id() == 0) {
    s_off = 0;
    s_slot = 0;
  }
  __syncthreads();
  unsigned long long acc = 0;
  int cnt = 0;
  for (int k = threadIdx.x; k < b; k += blockDim.x) {
    const int n = p.lens[k];
    acc += (unsigned long long)n;
    cnt += n > rows ? 1 : 0;
  }
  atomicAdd(&s_off, acc);
  atomicAdd(&s_slot, cnt);
  __syncthreads();
  const QueryPos qp{uniform_i64(s_off), __builtin_amdgcn_readfirstlane(s_slot)};
  __syncthreads();
  return qp;
}

__device__ __forceinline__ int64_t query_offset(const FwdParams& p, int b) {
  return query_pos(p, b, 0x7fffffff).off;
}

// The same for a one-wavefront team that shares its workgroup with others:
// a wavefront sum, no LDS and no workgroup barrier.
__device__ __forceinline__ int64_t wave_query_offset(const FwdParams& p, int b) {
  if (p.offsets != nullptr) return p.offsets[b];
  unsigned long long acc = 0;
  for (int k = (int)(threadIdx.x & (kWave - 1)); k < b; k += kWave)
    acc += (unsigned long long)p.lens[k];
  for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  return uniform_i64(acc);
}

// One workgroup per query; a query longer than one pass owns the row-buffer
// slot of its rank among such queries.
template <int R, int T, int W, int KS, int XL, int KIND, bool CKPT>
__global__ __launch_bounds__(kWave * W) void sdtw_fwd_kernel(const FwdParams p) {
  using S = FwdShape<R, T, W, KS, XL>;
  __shared__ __attribute__((aligned(16))) float s_mem[S::template lds_floats<CKPT>()];
  const int b = blockIdx.x;
  const QueryPos qp = query_pos(p, b, S::ROWS);
  float* row = p.rowbuf + (int64_t)qp.slot * p.row_stride;
  fwd_query<R, T, W, KS, XL, KIND, CKPT>(p, b, qp.off, row, s_mem);
}

// Binary16 form: one workgroup per pair of queries (2i, 2i+1), which must
// have equal lengths; an odd batch's last query fills both halves.  Each
// pair owns one row-buffer slot.
template <int R, int T, int W, int KS, int XL, int KIND>
__global__ __launch_bounds__(kWave * W) void sdtw_fwd16_kernel(const FwdParams p) {
  using S = FwdShape<R, T, W, KS, XL>;
  __shared__ __attribute__((aligned(16))) float s_mem[S::LDS_FLOATS];
  const int b = 2 * (int)blockIdx.x;
  float* row = p.rowbuf + (int64_t)blockIdx.x * p.row_stride;
  fwd_query<R, T, W, KS, XL, KIND, false, f16x2>(p, b, query_offset(p, b), row, s_mem);
}

// uint8-code form (binary32 DP of quantised values): one workgroup per query;
// queries and reference hold one code byte per element.
template <int R, int T, int W, int KS, int XL>
__global__ __launch_bounds__(kWave * W) void sdtw_fwd_u8_kernel(const FwdParams p) {
  using S = FwdShape<R, T, W, KS, XL>;
  __shared__ __attribute__((aligned(16))) float s_mem[S::LDS_FLOATS];
  const int b = blockIdx.x;
  float* row = p.rowbuf + (int64_t)b * p.row_stride;
  fwd_query<R, T, W, KS, XL, kSquared, false, Code8>(p, b, query_offset(p, b), row, s_mem);
}

// Persistent form: a fixed grid of teams pops queries (in the given order,
// longest first) from a device counter; each team owns one row-buffer slot
// (for queries that need several passes) and its own LDS.  A workgroup
// holds persistent_teams(W) teams: four independent one-wavefront teams for
// W = 1 (a grid of one-wavefront workgroups was placed unevenly on the
// SIMDs), else one.  Every team leaves the loop once the counter passes
// the batch size.
template <int R, int T, int W, int KS, int XL, int KIND, bool CKPT>
__global__ __launch_bounds__(kWave * W * persistent_teams(W)) void sdtw_fwd_persistent_kernel(
    const FwdParams p) {
  using S = FwdShape<R, T, W, KS, XL>;
  constexpr int TEAMS = persistent_teams(W);
  constexpr int TEAM_FLOATS = S::template lds_floats<CKPT>();
  __shared__ __attribute__((aligned(16))) float s_mem[TEAM_FLOATS * TEAMS];
  __shared__ int s_item;
  const int team = TEAMS > 1 ? wave_id() : 0;
  float* row = p.rowbuf + ((int64_t)blockIdx.x * TEAMS + team) * p.row_stride;
  float* mem = s_mem + team * TEAM_FLOATS;
  // The team's wave 0 pops the next item: every lane takes part in the
  // atomic (lane 0 adds 1, the others 0) so there is no lane-dependent
  // branch; with several waves the value is broadcast through LDS.  The
  // item is made wave-uniform with readfirstlane, so the loop, which holds
  // barriers, has a uniform exit.
  const int lane = threadIdx.x & (kWave - 1);
  for (;;) {
    int item;
    if constexpr (W == 1) {
      item = __builtin_amdgcn_readfirstlane(atomicAdd(p.queue, lane == 0 ? 1 : 0));
    } else {
      if (wave_id() == 0) {
        const int old = atomicAdd(p.queue, lane == 0 ? 1 : 0);
        s_item = __builtin_amdgcn_readfirstlane(old);
      }
      __syncthreads();
      item = __builtin_amdgcn_readfirstlane(s_item);
      __syncthreads();
    }
    if (item >= p.batch) break;
    const int b = __builtin_amdgcn_readfirstlane(p.order[item]);
    const int64_t off = TEAMS > 1 ? wave_query_offset(p, b) : query_offset(p, b);
    // a query's last pass may hold fewer rows per lane (not with checkpoints)
    fwd_query<R, T, W, KS, XL, KIND, CKPT, float, CKPT ? R : tail_rows_min<R>()>(
        p, b, off, row, mem);
  }
}

}  // namespace sdtw
