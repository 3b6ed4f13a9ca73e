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
constexpr int kWalkChunk = 32;                  // code rows per walker LDS chunk
constexpr int kBwdMaxSlots = 8;                 // blocks per round per query

// Direction code of a cell, 2 bits: a = "the diagonal is not a minimum",
// u = "the cell above is not a minimum".  The walk steps diagonally if a is
// clear, else up if u is clear, else left (ties: diagonal, then up, then
// left).  A lane's 16 cells of a row fill one word from the top: cell c's a
// is bit 2(15-c)+1 and its u is bit 2(15-c).
//
// Shift "x is not a minimum" into the word from below.  For x >= mn the
// binary32 difference mn - x has its sign bit set exactly when x != mn: it is
// +0 for equal values (an exact zero difference rounds to +0), negative or -0
// otherwise (a difference of distinct finite values is never +0), -inf for
// x = +inf > mn, and a positive NaN for x = mn = +inf.  v_alignbit_b32 then
// forms (word << 1) | (that sign bit).  The subtraction is an FP32 VALU
// instruction, which gfx950 dual-issues far more readily than an integer one.
__device__ __forceinline__ uint32_t push_not_min(uint32_t word, float x, float mn) {
  const float d = mn - x;
  return __builtin_amdgcn_alignbit(word, __builtin_bit_cast(uint32_t, d), 31);
}

struct BwdParams {
  const float* queries;       // packed
  const int32_t* lens;        // [batch]
  const int64_t* offsets;     // [batch + 1]
  const float* reference;     // [ref_len]
  const float* grad_cost;     // [batch]
  const float* cost;          // [batch], the forward's
  const int64_t* end_pos;     // [batch]
  const float* ckpt;          // forward checkpoints (nullptr when n_ckpt == 0)
  const float* rowck;         // the forward's row checkpoints (nullptr when n_ckpt == 0)
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
  int32_t max_rows;           // longest query (sizes the LDS of the kernels)
  int32_t round;
  int32_t nband;              // row bands per recomputed block (1: the whole block;
                              // 0 in a round kernel with no round after it)
  int32_t band_rows;          // rows of a band (a multiple of kRowCkpt) when nband > 1
  int64_t code_half;          // words of one code buffer (two alternate by round)
};

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t wave_uniform64(int64_t v) {
  const unsigned long long u = (unsigned long long)v;
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(u >> 32));
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(u & 0xffffffffu));
  return (int64_t)(((unsigned long long)hi << 32) | lo);
}

// Codes of segment s of round slot t of query b in the code buffer of round
// r (rounds alternate between two buffers): n + 63 rows of 64 words; word l
// of row g holds the 16 codes of lane l at step g, i.e. of query row
// i = g - l + 1 and columns 16l .. 16l+15 of the segment.  Rows of all the
// query's segments of a round are interleaved (row g of every segment, then
// row g+1, ...; code_row_stride words apart), so the wavefronts recomputing
// one query's blocks side by side write one contiguous stream per step.
__device__ __forceinline__ int64_t code_row_stride(const BwdParams& p) {
  return (int64_t)p.slots * p.nseg * kWave;
}

__device__ __forceinline__ int64_t code_segment(const BwdParams& p, int r, int b, int64_t qoff,
                                                int t, int s) {
  const int64_t base = code_row_stride(p) * (qoff + (int64_t)(kWave - 1) * b);
  return (r & 1) * p.code_half + base + ((int64_t)t * p.nseg + s) * kWave;
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

// Start of each query's path (the column of its row-1 cell), widened to the
// ABI's index type.
__global__ __launch_bounds__(kInitThreads) void sdtw_align_start_kernel(
    const int32_t* __restrict__ path_lo, int32_t batch, int64_t* __restrict__ start_pos) {
  const int b = blockIdx.x * kInitThreads + threadIdx.x;
  if (b < batch) start_pos[b] = path_lo[b];
}

// Lane 0's inputs of step g (row g+1): the segment's left column and the
// query value, read one step ahead of their use.
__device__ __forceinline__ void dirs_inputs(int g, int nrows, const float* lq, const float* ledge,
                                            float& il, float& iq) {
  const int gi = g < nrows ? g : nrows - 1;
  il = ledge[gi];
  iq = lq[gi];
}

// One row step of the direction recompute.  MASKED: some lanes are outside
// rows 1..nrows and keep their state (row 0 before they start).
template <int KIND, bool MASKED>
__device__ __forceinline__ void dirs_step(int g, int lane, int nrows, float il, float iq,
                                          float* ledge, const float (&rv)[kDirCols],
                                          float (&dprev)[kDirCols], float& last, float& shp,
                                          float& qv, uint32_t* __restrict__ out, int64_t rs) {
  const float shc = wave_shr1(il, last);          // left neighbour on this row
  qv = wave_shr1(iq, qv);                         // this row's query value
  float cur[kDirCols];
  uint32_t word = 0;
  float left = shc, diag = shp;
#pragma unroll
  for (int c = 0; c < kDirCols; ++c) {
    const float up = dprev[c];
    const float mn = min3(up, left, diag);
    word = push_not_min(word, diag, mn);
    word = push_not_min(word, up, mn);
    cur[c] = mn + local_cost<KIND>(qv, rv[c]);
    diag = up;
    left = cur[c];
  }
  const int i = g - lane + 1;
  // (a lane outside rows 1..nrows stores nothing: with row bands, those
  // code words belong to the neighbouring band)
  if (!MASKED || (i >= 1 && i <= nrows)) {
    // (non-temporal: codes are written once and most are never read, so
    // they should not displace, or leave dirty, cache lines other kernels use)
    __builtin_nontemporal_store(word, &out[(int64_t)g * rs]);
#pragma unroll
    for (int c = 0; c < kDirCols; ++c) dprev[c] = cur[c];
    last = cur[kDirCols - 1];
    // right column of this segment = left column of the next one; entry
    // i-1 was read by lane 0 at step i-1, 63 steps earlier
    if (lane == kWave - 1) ledge[i - 1] = last;
  }
  shp = shc;
}

// Recompute rows 1..i of block slot t of round r of query b (i = the
// walker's current row as last stored, which only decreases, so any value
// read is enough; lowered further by the block's right checkpoint column)
// and store its direction codes.  With p.nband > 1 the block is split into
// bands of p.band_rows rows, each recomputed on its own from the forward's
// row checkpoint above it; this call takes band z.  One wavefront; LDS
// `dyn`: query values and the left boundary column, 2 * max_rows floats.
template <int KIND>
__device__ __forceinline__ void dirs_block(const BwdParams& p, int r, int b, int t, int z,
                                           float* dyn) {
  const int lane = threadIdx.x & (kWave - 1);
  if (wave_uniform(p.state[4 * b + 2]) != 0) return;
  const int K = p.ckpt_every;
  const int64_t e = wave_uniform64(p.end_pos[b]);
  const int blk_end = (int)(e / K);
  const int blk = blk_end - r * p.slots - t;
  if (blk < 0) return;
  const int n = wave_uniform(p.lens[b]);
  int nrows = wave_uniform(p.state[4 * b + 0]);
  const int64_t qoff = wave_uniform64(p.offsets[b]);
  if (blk < blk_end) {
    // D never decreases along the path, so the cell where the walk enters
    // this block (in its last column, which checkpoint blk+1 holds) has
    // D <= cost: rows below the last such row are not needed.
    const float* ckr = p.ckpt + qoff * p.n_ckpt + (int64_t)blk * n;
    const float cost = p.cost[b];
    int last = 0;
    for (int k = lane; k < nrows; k += kWave)
      if (ckr[k] <= cost) last = k + 1;
    for (int off = kWave / 2; off > 0; off >>= 1) {
      const int o = __shfl_xor(last, off);
      last = o > last ? o : last;
    }
    nrows = wave_uniform(last);
    if (nrows == 0) return;                    // the path does not reach this block
  }
  // band z: rows r0+1 .. r0+brows (r0 a multiple of kRowCkpt)
  const int r0 = z * p.band_rows;
  if (r0 >= nrows) return;
  const int brows = p.nband > 1 && r0 + p.band_rows < nrows ? p.band_rows : nrows - r0;
  float* lq = dyn;
  float* ledge = dyn + p.max_rows;
  const float* __restrict__ q = p.queries + qoff + r0;
  const float* ck = blk > 0 ? p.ckpt + qoff * p.n_ckpt + (int64_t)(blk - 1) * n + r0 : nullptr;
  for (int k = lane; k < brows; k += kWave) {
    lq[k] = q[k];
    ledge[k] = blk > 0 ? ck[k] : inf_f32();
  }
  // (the LDS region is this wavefront's own: a wavefront-level barrier)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // the band's top boundary: row r0 (row 0 = zeros for the first band)
  const float* top =
      r0 > 0 ? p.rowck + (qoff / kRowCkpt + r0 / kRowCkpt - 1) * (int64_t)p.ref_len : nullptr;

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
    // band-local step g stores code row r0 + g
    const int64_t rs = code_row_stride(p);
    uint32_t* out = p.codes + code_segment(p, r, b, qoff, t, s) + (int64_t)r0 * rs + lane;
    // Row r0 of the segment's columns; a lane's `last` is its right-most
    // value there (lane l+1's diagonal for its first row), and lane 0's
    // first diagonal is D(r0, cs-1) (+inf left of column 1 below row 0).
    float dprev[kDirCols];
    float shp = 0.0f;
    if (top != nullptr) {
#pragma unroll
      for (int c = 0; c < kDirCols; ++c) {
        const int j = cs + lane * kDirCols + c;
        dprev[c] = j < p.ref_len ? top[j] : 0.0f;
      }
      shp = cs > 0 ? top[cs - 1] : inf_f32();
    } else {
#pragma unroll
      for (int c = 0; c < kDirCols; ++c) dprev[c] = 0.0f;    // row 0
    }
    float last = dprev[kDirCols - 1], qv = 0.0f;
    const int g_end = brows + kWave - 1;
    const int g_head = g_end < kWave - 1 ? g_end : kWave - 1;
    // (lane 63 writes ledge[g-63] at step g, long after it was read)
    float ilA, iqA, ilB, iqB;
    dirs_inputs(0, brows, lq, ledge, ilA, iqA);
    int g = 0;
    for (; g < g_head; ++g) {
      dirs_inputs(g + 1, brows, lq, ledge, ilB, iqB);
      dirs_step<KIND, true>(g, lane, brows, ilA, iqA, ledge, rv, dprev, last, shp, qv, out, rs);
      ilA = ilB;
      iqA = iqB;
    }
    for (; g + 1 < brows; g += 2) {
      dirs_inputs(g + 1, brows, lq, ledge, ilB, iqB);
      dirs_step<KIND, false>(g, lane, brows, ilA, iqA, ledge, rv, dprev, last, shp, qv, out,
                             rs);
      dirs_inputs(g + 2, brows, lq, ledge, ilA, iqA);
      dirs_step<KIND, false>(g + 1, lane, brows, ilB, iqB, ledge, rv, dprev, last, shp, qv,
                             out, rs);
    }
    for (; g < g_end; ++g) {
      dirs_inputs(g + 1, brows, lq, ledge, ilB, iqB);
      dirs_step<KIND, true>(g, lane, brows, ilA, iqA, ledge, rv, dprev, last, shp, qv, out, rs);
      ilA = ilB;
      iqA = iqB;
    }
  }
}

// Code rows [kWalkChunk * k, kWalkChunk * (k + 1)) of a segment (rs words
// apart) staged as kWalkChunk * 64 consecutive words; each lane holds
// kWalkChunk / 4 uint4 of them.  Rows past the segment's end read as zero
// (they are never addressed).
struct CodeChunk {
  uint4 v[kWalkChunk * kWave / (4 * kWave)];

  __device__ __forceinline__ void fetch(const uint32_t* seg, int64_t rs, int k, int code_rows,
                                        int lane) {
#pragma unroll
    for (int u = 0; u < kWalkChunk / 4; ++u) {
      const int e = 4 * (lane + kWave * u);             // word within the chunk
      const int row = k * kWalkChunk + e / kWave;
      v[u] = row < code_rows
                 ? *reinterpret_cast<const uint4*>(seg + (int64_t)row * rs + (e & (kWave - 1)))
                 : make_uint4(0u, 0u, 0u, 0u);
    }
  }
  __device__ __forceinline__ void commit(uint32_t* lds, int lane) const {
#pragma unroll
    for (int u = 0; u < kWalkChunk / 4; ++u)
      *reinterpret_cast<uint4*>(lds + 4 * (lane + kWave * u)) = v[u];
  }
};

// Follow the direction codes of round r's blocks of query b.  One wavefront;
// every lane runs the same (uniform) walk.  Code rows are staged through LDS
// (`chunk`, kWalkChunk rows) kWalkChunk at a time: within a segment the code
// row g = i - 1 + (lane owning column j) never increases along the walk, so
// the chunk below the current one is always the next one needed and is
// fetched ahead.
__device__ __forceinline__ void walk_query(const BwdParams& p, int r, int b, uint32_t* chunk) {
  const int lane = threadIdx.x & (kWave - 1);
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
  const int64_t rs = code_row_stride(p);
  int done = 0;

  for (int t = 0; t < p.slots && !done; ++t) {
    const int blk = blk_end - r * p.slots - t;
    if (blk < 0) break;
    const int bc0 = blk * K;
    for (int s = (j - bc0) / kDirSeg; s >= 0 && !done; --s) {
      const int cs = bc0 + s * kDirSeg;
      const uint32_t* seg = p.codes + code_segment(p, r, b, qoff, t, s);
      CodeChunk pre;                            // the chunk fetched ahead
      int kc = -1, kp = -1;                     // chunk in LDS, chunk in `pre`
      while (j >= cs) {
        const int L = (j - cs) >> 4;
        const int c = (j - cs) & (kDirCols - 1);
        const int g = i - 1 + L;                // >= 0: i >= 1, L >= 0
        const int k = (int)((unsigned)g / kWalkChunk);
        if (k != kc) {
          if (kp != k) pre.fetch(seg, rs, k, code_rows, lane);
          __builtin_amdgcn_wave_barrier();
          pre.commit(chunk, lane);
          __builtin_amdgcn_wave_barrier();
          kc = k;
          kp = k - 1;
          if (k > 0) pre.fetch(seg, rs, k - 1, code_rows, lane);
        }
        const uint32_t w =
            (uint32_t)wave_uniform((int)chunk[((unsigned)g % kWalkChunk) * kWave + L]);
        // pass through the cells c, c-1, ... of this word whose code is
        // "left" (cell c' is bit pair 15-c'); the first other one ends the
        // run in this row
        const uint32_t is_left = (w >> 1) & w & 0x55555555u;   // at bit 2(15-c')
        const int pc = kDirCols - 1 - c;
        const uint32_t stop = ~is_left & 0x55555555u & (~0u << (2 * pc));
        if (stop == 0) {
          // The rest of this word is "left", so the run goes on in the words
          // of lanes L-1, L-2, ... of row i, which sit on a diagonal of the
          // staged rows (lane x's word at code row g - (L - x)).  Every lane
          // x in [xlo, L) whose word is in this chunk tests its own word at
          // once; a ballot finds the right-most one holding a cell that is
          // not "left", and the walk continues at that word's last column,
          // or below the chunk if there is none.
          const int d0 = g - kc * kWalkChunk;   // chunk row of the current word
          const int xlo = L > d0 ? L - d0 : 0;
          const bool mine = lane >= xlo && lane < L;
          const uint32_t wx = chunk[(mine ? d0 - L + lane : 0) * kWave + lane];
          const bool stops = mine && (((wx >> 1) & wx & 0x55555555u) != 0x55555555u);
          const unsigned long long m = __ballot(stops);
          j = m != 0 ? cs + kDirCols * (kWave - 1 - __clzll(m)) + (kDirCols - 1)
                     : cs + kDirCols * xlo - 1;
          continue;
        }
        const int bit = __builtin_ctz(stop);    // 2(15-c') for the cell c' that stops
        j -= (bit >> 1) - pc;
        // (every lane stores the same value to the same address: one write,
        // and no lane mask to set up and restore around it)
        if (i == 1) {                           // the start cell
          rlo[1] = j;
          p.path_lo[b] = j;
          done = 1;
          break;
        }
        const bool diagonal = ((w >> (bit + 1)) & 1u) == 0;
        rlo[i] = j;
        i -= 1;
        if (diagonal) j -= 1;
        rhi[i] = j;
      }
    }
  }
  if (lane == 0) {
    p.state[4 * b + 0] = i;
    p.state[4 * b + 1] = j;
    p.state[4 * b + 2] = done;
  }
}

// LDS of one round-kernel wavefront: the larger of the walker's code chunk
// and the dirs block's query + left column.
__host__ __device__ constexpr size_t bwd_round_lds_bytes(int max_rows) {
  return sizeof(float) * 2 * (size_t)max_rows > sizeof(uint32_t) * kWalkChunk * kWave
             ? sizeof(float) * 2 * (size_t)max_rows
             : sizeof(uint32_t) * kWalkChunk * kWave;
}

// Round 0's blocks, one wavefront each, blockDim.x / 64 wavefronts per
// workgroup (each with its own 2 * max_rows floats of LDS): block item
// e = blockIdx.x * (blockDim.x / 64) + wave is query e % batch, slot
// e / batch.  (Several wavefronts per workgroup keep the placement even: a
// grid of as many one-wavefront workgroups as two per SIMD was placed
// unevenly depending on the kernel before it, up to 1.4 times slower.)
template <int KIND>
__global__ __launch_bounds__(4 * kWave) void sdtw_bwd_dirs_kernel(const BwdParams p) {
  extern __shared__ __attribute__((aligned(16))) float dyn[];
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int e = (int)blockIdx.x * (int)(blockDim.x / kWave) + w;
  if (e >= p.batch * p.slots) return;
  dirs_block<KIND>(p, 0, e % p.batch, e / p.batch, 0, dyn + (size_t)w * 2 * p.max_rows);
}

// Round r = p.round: wavefronts [0, batch) walk round r; when another round
// follows, wavefronts [batch, batch + batch * slots * nband) recompute round
// r+1's blocks (row bands) into the other code buffer meanwhile.  Wavefront
// e = blockIdx.x * (blockDim.x / 64) + wave, each with its own
// bwd_round_lds_bytes(max_rows) of LDS (several wavefronts per workgroup
// keep the placement on the SIMDs even).
template <int KIND>
__global__ __launch_bounds__(4 * kWave) void sdtw_bwd_round_kernel(const BwdParams p) {
  extern __shared__ __attribute__((aligned(16))) float dyn[];
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int x = (int)blockIdx.x * (int)(blockDim.x / kWave) + w;
  float* mine = dyn + (size_t)w * (bwd_round_lds_bytes(p.max_rows) / sizeof(float));
  if (x < p.batch) {
    walk_query(p, p.round, x, reinterpret_cast<uint32_t*>(mine));
  } else {
    const int k = x - p.batch;
    const int tz = k / p.batch;
    if (tz < p.slots * p.nband)
      dirs_block<KIND>(p, p.round + 1, k % p.batch, tz / p.nband, tz % p.nband, mine);
  }
}

// Gradients from the recorded path rows.  Grid: (batch, RG + kGradColGroups),
// RG = ceil(max_rows / kGradThreads), kGradThreads threads.  blockIdx.y = y
// < RG takes the query sums of rows y*kGradThreads + 1 .., one thread per row
// (dispatched first: their longest runs are the kernel's longest chains);
// blockIdx.y = RG + g takes the reference partials of share g of
// kGradColGroups equal shares of the query's column span, with the row
// bounds (2 * max_rows ints) and, with QLDS, the query values (max_rows
// floats) in dynamic LDS.  Row i's path
// columns are [row_lo[i], row_hi[i]];
// both bounds are nondecreasing in i, so the rows of column j are the run
// from its top row (the first row with row_hi >= j) down to its bottom row
// (the last row with row_lo <= j).
//   grad_q[i]      = sum over row i's columns j (descending) of g*dc/dq;
//   ref_part[b][j] = sum over column j's rows i (descending) of -g*dc/dq,
//                    for j in [path_lo, end_pos], each thread a contiguous
//                    range of columns, following the top row along it.
// Reference values are loaded in batches, the next batch while the current
// one is summed.
constexpr int kGradThreads = 256;
constexpr int kGradColGroups = 8;               // workgroups per query for column sums
constexpr int kGradBatch = 8;                   // column sums
constexpr int kGradRowBatch = 16;               // row sums from global memory
constexpr int kGradRowBatchLds = 16;            // row sums from LDS

constexpr int kGradRowLds = 8192;               // reference values a row group stages

__host__ __device__ constexpr bool bwd_grad_q_in_lds(int max_rows) {
  return sizeof(int32_t) * 3 * (size_t)max_rows <= 65536;
}

__host__ __device__ constexpr size_t bwd_grad_lds_bytes(int max_rows) {
  return sizeof(int32_t) * (bwd_grad_q_in_lds(max_rows) ? 3 : 2) * (size_t)max_rows >
                 sizeof(float) * (size_t)kGradRowLds
             ? sizeof(int32_t) * (bwd_grad_q_in_lds(max_rows) ? 3 : 2) * (size_t)max_rows
             : sizeof(float) * (size_t)kGradRowLds;
}

// grad_q[i] of one row: the run of columns hi, hi-1, .., lo (src[j - off]
// is the reference value of column j), added in that order.  Whole batches
// of B columns are read at fixed offsets from one pointer, the next batch
// while the current one is added, into two register sets used in turn (at
// the last whole batch the "next" read repeats the current one, which stays
// in bounds); the fewer than B columns left are added one by one.
template <int KIND, int B>
__device__ __forceinline__ void row_batch(float& acc, float qi, float gcost, const float (&v)[B]) {
#pragma unroll
  for (int u = 0; u < B; ++u) acc = acc + gcost * dcost_dq<KIND>(qi, v[u]);
}

template <int B>
__device__ __forceinline__ void row_load(float (&v)[B], const float* s) {
#pragma unroll
  for (int u = 0; u < B; ++u) v[u] = s[-u];
}

template <int KIND, int B>
__device__ __forceinline__ float row_sum(const float* __restrict__ src, int off, float qi,
                                         float gcost, int lo, int jj) {
  float acc = 0.0f;
  const float* s = src + (jj - off);            // column jj
  const int full = (jj - lo + 1) / B;
  float va[B], vb[B];
  if (full > 0) row_load<B>(va, s);
  int k = 0;
  for (; k + 1 < full; k += 2) {                // batches k (in va) and k+1
    row_load<B>(vb, s - B);
    row_batch<KIND, B>(acc, qi, gcost, va);
    s -= B;
    row_load<B>(va, k + 2 < full ? s - B : s);
    row_batch<KIND, B>(acc, qi, gcost, vb);
    s -= B;
  }
  if (k < full) {                               // the last whole batch, in va
    row_batch<KIND, B>(acc, qi, gcost, va);
    s -= B;
  }
  // the columns left: s[0], s[-1], .. down to column lo
  const int rem = (jj - lo + 1) - full * B;
  for (int u = 0; u < rem; ++u) acc = acc + gcost * dcost_dq<KIND>(qi, s[-u]);
  return acc;
}

__host__ __device__ constexpr int bwd_grad_row_groups(int max_rows) {
  return (max_rows + kGradThreads - 1) / kGradThreads;
}

__device__ __forceinline__ int clamp_col(int v, int lo, int hi) {
  return v > lo ? (v < hi ? v : hi) : lo;
}

template <int KIND, bool QLDS>
__global__ __launch_bounds__(kGradThreads) void sdtw_bwd_grad_kernel(const BwdParams p) {
  extern __shared__ int32_t dyn_rows[];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int n = p.lens[b];
  const int64_t qoff = p.offsets[b];
  const float* __restrict__ r = p.reference;
  const float gcost = p.grad_cost[b];
  // (the clamps only keep every access in bounds; a finished walk records
  // every row, with columns in [path_lo, end_pos])
  const int jhi = (int)p.end_pos[b];
  const int jlo = p.path_lo[b] > 0 ? (p.path_lo[b] < jhi ? p.path_lo[b] : jhi) : 0;

  const int row_groups = bwd_grad_row_groups(p.max_rows);
  if ((int)blockIdx.y < row_groups) {
    // rows i0 .. i0+255: row bounds never decrease with the row, so their
    // columns are the one span [lo(i0), hi(last row)], staged in LDS when it
    // fits (values left of a row's lo are loaded but never added)
    const int i0 = blockIdx.y * kGradThreads + 1;
    if (i0 > n) return;
    const int ilast = i0 + kGradThreads - 1 < n ? i0 + kGradThreads - 1 : n;
    const int slo = clamp_col(p.row_lo[qoff + i0 - 1], jlo, jhi);
    const int shi = clamp_col(p.row_hi[qoff + ilast - 1], jlo, jhi);
    const bool staged = shi - slo < kGradRowLds;
    float* lr = reinterpret_cast<float*>(dyn_rows);
    if (staged) {
      for (int e = tid; e <= shi - slo; e += kGradThreads) lr[e] = r[slo + e];
      __syncthreads();
    }
    const int i = i0 + tid;
    if (i > n) return;
    const float qi = p.queries[qoff + i - 1];
    const int lo = clamp_col(p.row_lo[qoff + i - 1], jlo, jhi);
    const int hi = clamp_col(p.row_hi[qoff + i - 1], jlo, jhi);
    p.grad_q[qoff + i - 1] = staged ? row_sum<KIND, kGradRowBatchLds>(lr, slo, qi, gcost, lo, hi)
                                    : row_sum<KIND, kGradRowBatch>(r, 0, qi, gcost, lo, hi);
    return;
  }

  float* __restrict__ part = p.ref_part + (int64_t)b * p.part_stride;
  int32_t* rlo = dyn_rows - 1;                  // indexed by 1-based row
  int32_t* rhi = dyn_rows + p.max_rows - 1;
  float* lq = reinterpret_cast<float*>(dyn_rows + 2 * p.max_rows);
  for (int i = 1 + tid; i <= n; i += kGradThreads) {
    rlo[i] = clamp_col(p.row_lo[qoff + i - 1], jlo, jhi);
    rhi[i] = clamp_col(p.row_hi[qoff + i - 1], jlo, jhi);
    if constexpr (QLDS) lq[i - 1] = p.queries[qoff + i - 1];
  }
  __syncthreads();
  const float* __restrict__ q = QLDS ? lq : p.queries + qoff;

  const int span = jhi - jlo + 1;
  const int per = (span + kGradColGroups * kGradThreads - 1) / (kGradColGroups * kGradThreads);
  const int j0 = jlo + ((blockIdx.y - row_groups) * kGradThreads + tid) * per;
  const int j1 = j0 + per < jhi + 1 ? j0 + per : jhi + 1;
  if (j0 < j1) {
    int a = 1, z = n;                           // top row of column j0
    while (a < z) {
      const int mid = (a + z) >> 1;
      if (rhi[mid] >= j0) z = mid; else a = mid + 1;
    }
    int top = a;
    float qtop = q[top - 1];
    for (int jb = j0; jb < j1; jb += kGradBatch) {
      float rv[kGradBatch];
#pragma unroll
      for (int u = 0; u < kGradBatch; ++u) rv[u] = jb + u < j1 ? r[jb + u] : 0.0f;
#pragma unroll
      for (int u = 0; u < kGradBatch; ++u) {
        const int jj = jb + u;
        if (jj < j1) {
          // top row of column jj: the first row whose last column is >= jj
          // (last columns never decrease with the row), searched from the
          // previous column's top row by doubling steps, then bisection
          // (a steep stretch of the path moves it by many rows at once)
          if (top < n && rhi[top] < jj) {
            int a = top + 1, z = top + 1, step = 1;
            while (z < n && rhi[z] < jj) {
              a = z + 1;
              z = z + step < n ? z + step : n;
              step <<= 1;
            }
            while (a < z) {
              const int mid = (a + z) >> 1;
              if (rhi[mid] >= jj) z = mid; else a = mid + 1;
            }
            top = a;
            qtop = q[top - 1];
          }
          // bottom row of column jj: the last row whose first column is <= jj
          // (first columns never decrease with the row; a binary search for
          // the rare vertical runs)
          int bottom = top;
          if (bottom < n && rlo[bottom + 1] <= jj) {
            int a = bottom + 1, z = n;
            while (a < z) {
              const int mid = (a + z + 1) >> 1;
              if (rlo[mid] <= jj) a = mid; else z = mid - 1;
            }
            bottom = a;
          }
          // rows bottom, bottom-1, .., top, query values read 8 at a time
          float acc = 0.0f;
          int ii = bottom;
          for (; ii - 7 > top; ii -= 8) {
            float qv[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) qv[v] = q[ii - v - 1];
#pragma unroll
            for (int v = 0; v < 8; ++v) acc = acc + (-(gcost * dcost_dq<KIND>(qv[v], rv[u])));
          }
          for (; ii > top; --ii) acc = acc + (-(gcost * dcost_dq<KIND>(q[ii - 1], rv[u])));
          part[jj] = acc + (-(gcost * dcost_dq<KIND>(qtop, rv[u])));
        }
      }
    }
  }
}

// grad_reference[j] = sum over queries b (increasing) whose path covers
// column j of ref_part[b][j]; +0 where no path passes.  Only entries inside
// a query's span [path_lo, end_pos] are loaded (the others were never
// written) and the rest read as +0; the running sum starts at +0 and is
// never -0, so adding +0 leaves it unchanged and the result equals the sum
// over covering queries only.  Queries go 64 at a time: each wavefront
// loads their spans with one vector load per bound (one query per lane) and
// reads them back with readlane, and loads the next 64 queries' entries
// while it adds the current ones.
constexpr int kRefReduceThreads = 256;
constexpr int kRefReduceBatch = kWave;

struct RefSpans {
  int lo, hi;           // span of query b0 + lane (empty past the batch)

  __device__ __forceinline__ void load(const int32_t* __restrict__ path_lo,
                                       const int64_t* __restrict__ end_pos, int32_t batch,
                                       int b0, int lane) {
    const int b = b0 + lane;
    lo = b < batch ? path_lo[b] : 1;
    hi = b < batch ? (int)end_pos[b] : 0;
  }
};

__device__ __forceinline__ void ref_part_batch(const float* __restrict__ ref_part,
                                               int64_t part_stride, const RefSpans& sp, int b0,
                                               int j, float (&v)[kRefReduceBatch]) {
#pragma unroll
  for (int u = 0; u < kRefReduceBatch; ++u) {
    const int l = __builtin_amdgcn_readlane(sp.lo, u);
    const int h = __builtin_amdgcn_readlane(sp.hi, u);
    v[u] = j >= l && j <= h ? ref_part[(int64_t)(b0 + u) * part_stride + j] : 0.0f;
  }
}

__global__ __launch_bounds__(kRefReduceThreads) void sdtw_ref_reduce_kernel(
    const float* __restrict__ ref_part, int64_t part_stride, const int32_t* __restrict__ lo,
    const int64_t* __restrict__ hi, int32_t batch, int32_t ref_len, float* __restrict__ grad_ref) {
  const int lane = threadIdx.x & (kWave - 1);
  const int j = blockIdx.x * kRefReduceThreads + threadIdx.x;
  // (lanes past ref_len stay in the loop, whose bounds are uniform, and
  // load nothing: no span reaches them)
  float acc = 0.0f;
  float v[kRefReduceBatch], nv[kRefReduceBatch];
  RefSpans sp;
  sp.load(lo, hi, batch, 0, lane);
  ref_part_batch(ref_part, part_stride, sp, 0, j, nv);
  for (int b = 0; b < batch; b += kRefReduceBatch) {
#pragma unroll
    for (int u = 0; u < kRefReduceBatch; ++u) v[u] = nv[u];
    if (b + kRefReduceBatch < batch) {
      sp.load(lo, hi, batch, b + kRefReduceBatch, lane);
      ref_part_batch(ref_part, part_stride, sp, b + kRefReduceBatch, j, nv);
    }
#pragma unroll
    for (int u = 0; u < kRefReduceBatch; ++u) acc = acc + v[u];
  }
  if (j < ref_len) grad_ref[j] = acc;
}

}  // namespace sdtw
