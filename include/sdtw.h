/*
 * sdtw.h -- C ABI of the MI355X subsequence dynamic time warping library
 * (libsdtw.so, built from paper_2403_06931_amd/csrc).
 *
 * Operation (paper: Section 2, Eq. (1) and the paragraph after it).  For a
 * query q of length N (DP rows i = 1..N) and a reference r of length M (DP
 * columns j = 1..M):
 *
 *     D(0,j) = 0 (j = 0..M),  D(i,0) = +inf (i = 1..N),
 *     D(i,j) = min{D(i-1,j), D(i,j-1), D(i-1,j-1)} + c(q_i, r_j),
 *
 * with c(q,r) = (q - r)^2 (SDTW_COST_SQUARED) or |q - r| (SDTW_COST_ABSOLUTE),
 * each operation in binary32 rounded to nearest-even, no fused multiply-add,
 * subnormals kept.  Per query the library returns
 *
 *     cost    = min_j D(N,j)
 *     end_pos = (smallest j attaining cost) - 1   (0-based, inclusive index of
 *               the reference element matched to the last query element).
 *
 * The batch form follows the paper's batched kernel (Section 5.2: many
 * queries stored back to back, no gaps, one result each); queries here may
 * have different lengths.
 *
 * Conventions shared by every entry point:
 *   - Pointers not prefixed h_ are DEVICE pointers owned by the caller.  The
 *     library keeps no pointer after a call returns and allocates no memory.
 *   - queries are packed float32: query b occupies
 *     [sum_{k<b} len_k, sum_{k<=b} len_k).
 *   - h_query_lens is a HOST copy of query_lens (device); the host copy drives
 *     validation, workspace sizing and scheduling, the device copy feeds the
 *     kernels.  They must hold the same values.
 *   - All work is enqueued on `stream` (a hipStream_t; NULL = the null
 *     stream) and is asynchronous; no call synchronises the device.
 *   - Arguments are validated on the host before any HIP call; an invalid
 *     call returns a negative status and enqueues nothing.  A kernel launch
 *     failure returns SDTW_ERR_HIP.  Faults inside kernels surface at the
 *     caller's next synchronisation.
 *   - Inputs containing NaN or infinity give unspecified results.
 *   - Concurrent calls that share a workspace race; use one workspace per
 *     stream.
 */
#ifndef SDTW_H
#define SDTW_H

#include <stddef.h>
#include <stdint.h>

#ifndef SDTW_API
#define SDTW_API __attribute__((visibility("default")))
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* Local cost d(q_i, r_j) (the paper leaves d open; Section 8 implies a
 * subtraction followed by a multiplication). */
enum {
    SDTW_COST_SQUARED = 0,
    SDTW_COST_ABSOLUTE = 1
};

/* Status codes. */
enum {
    SDTW_OK = 0,
    SDTW_ERR_INVALID_ARG = -1, /* null pointer, bad size, bad length, unknown cost kind */
    SDTW_ERR_WORKSPACE = -2,   /* workspace_bytes smaller than required */
    SDTW_ERR_UNSUPPORTED = -3, /* unknown variant, or a shape no compiled kernel covers */
    SDTW_ERR_HIP = -4          /* a HIP runtime call or kernel launch failed */
};

/* Flags for sdtw_forward. */
enum {
    /* Store DP column checkpoints for sdtw_backward (ckpt must be non-NULL). */
    SDTW_F_CHECKPOINT = 1,
    /* Persistent launch: a fixed grid of teams (W wavefronts each) pops
     * queries from a device work queue, longest first.  Meant for batches of
     * uneven lengths; the launch sequence is safe to capture in a HIP graph. */
    SDTW_F_PERSISTENT = 2
};

/* Size of the persistent grid, in flags bits 8..11: SDTW_F_WAVES_PER_SIMD(n)
 * asks for n resident wavefronts per SIMD (n = 1..8; 0 or absent: 2), i.e.
 * min(batch, CUs * 4 * n / W) teams of W wavefronts, four teams to a
 * workgroup when W = 1 (one otherwise).  Ignored without SDTW_F_PERSISTENT.
 * The grid size changes the workspace (one row-buffer slot per team of the
 * grid, rounded up to whole workgroups, when a query needs several passes),
 * never the results. */
#define SDTW_F_WAVES_SHIFT 8
#define SDTW_F_WAVES_MASK (0xf << SDTW_F_WAVES_SHIFT)
#define SDTW_F_WAVES_PER_SIMD(n) ((int32_t)(n) << SDTW_F_WAVES_SHIFT)

/* Largest accepted reference length (column indices are 32-bit inside the
 * kernels). */
#define SDTW_MAX_REF_LEN ((int64_t)1 << 30)

/*
 * Bytes of device workspace sdtw_forward needs for this batch, with `flags`
 * as passed to sdtw_forward and tile `variant` (-1: the variant the library
 * picks for this batch, as sdtw_forward does with variant -1).  Returns 0 on
 * invalid arguments or an unknown variant.
 * The workspace holds the offset and slot tables of large batches, the
 * persistent form's work counter and processing order, and a row buffer of
 * ceil(ref_len / 64) * 64 floats per slot that carries the last DP row of a
 * row pass to the next pass.  A pass covers 64 * R * W query rows (R rows per
 * lane, W wavefronts per query: sdtw_variant_info); the plain launch gives a
 * slot to each query longer than one pass, the persistent launch one to each
 * of its teams when some query is.  A batch whose queries all fit in
 * one pass needs no row buffer.  cost and end_pos are reduced on chip.
 */
SDTW_API size_t sdtw_forward_workspace_bytes(const int32_t *h_query_lens, int32_t batch,
                                    int64_t ref_len, int32_t flags, int32_t variant);

/*
 * Bytes of one workspace that serves every call of the differentiable path
 * on this batch: sdtw_forward with `flags` and the library's variant choice,
 * and, when flags has SDTW_F_CHECKPOINT, sdtw_backward and sdtw_align with
 * checkpoints every `ckpt_every` columns (the largest of their sizes; the
 * calls leave nothing in the workspace that a later call reads, so one
 * buffer can serve them in turn on one stream).  Returns 0 on invalid
 * arguments.
 */
SDTW_API size_t sdtw_workspace_bytes(const int32_t *h_query_lens, int32_t batch,
                                     int64_t ref_len, int32_t flags, int32_t ckpt_every);

/* Row-checkpoint spacing: the forward also stores D(k*256, 1..ref_len) for
 * every k >= 1 with k*256 < len_b, so that the backward can recompute a
 * block of columns as independent bands of 256 rows (or of a multiple of
 * 256 rows). */
#define SDTW_ROW_CKPT_EVERY 256

/*
 * Number of float32 entries of the checkpoint buffer for this batch and
 * checkpoint interval: n_ckpt * T + floor(T / 256) * ref_len, where
 * T = sum_b len_b and n_ckpt = ceil(ref_len / ckpt_every) - 1.
 * Layout, columns (Eq. (1)'s D over whole columns): query b's block starts
 * at offset(b) * n_ckpt (offset(b) = sum of the lengths of queries 0..b-1)
 * and holds n_ckpt columns of len_b values each; column k (k = 1..n_ckpt)
 * is D(1..len_b, k*ckpt_every), i.e. the DP column of 0-based reference
 * index k*ckpt_every - 1.
 * Then rows, from entry n_ckpt * T on: row r = floor(offset(b) / 256) + k - 1
 * of ref_len values is D(k*256, 1..ref_len) of query b, for k >= 1 and
 * k*256 < len_b (rows of different queries never coincide; rows no query
 * owns are left untouched).
 * Returns 0 if no checkpoint is needed (ref_len <= ckpt_every) or on invalid
 * arguments.
 */
SDTW_API size_t sdtw_checkpoint_floats(const int32_t *h_query_lens, int32_t batch,
                              int64_t ref_len, int32_t ckpt_every);

/*
 * Forward pass: cost[b] and end_pos[b] for every query.
 *
 *   queries      device float32, packed, sum(len) values
 *   h_query_lens host int32 [batch], every entry >= 1
 *   query_lens   device int32 [batch], same values
 *   batch        >= 1
 *   reference    device float32 [ref_len], 1 <= ref_len <= SDTW_MAX_REF_LEN
 *   cost_kind    SDTW_COST_SQUARED or SDTW_COST_ABSOLUTE
 *   cost         device float32 [batch]            (output)
 *   end_pos      device int64 [batch], 0-based     (output)
 *   ckpt         device float32 [sdtw_checkpoint_floats(...)] when flags has
 *                SDTW_F_CHECKPOINT (may be NULL if that count is 0), else
 *                ignored
 *   ckpt_every   checkpoint interval in reference columns, a positive
 *                multiple of 16, when checkpointing, else ignored
 *   variant      kernel tile variant (0 <= variant < sdtw_variant_count()),
 *                or -1 to let the library choose
 *   workspace    device, >= sdtw_forward_workspace_bytes(..., flags, variant)
 *                bytes, 256-byte aligned (SDTW_ERR_WORKSPACE if smaller)
 *   stream       hipStream_t or NULL
 */
SDTW_API int sdtw_forward(const float *queries, const int32_t *h_query_lens,
                 const int32_t *query_lens, int32_t batch,
                 const float *reference, int64_t ref_len, int32_t cost_kind,
                 float *cost, int64_t *end_pos,
                 float *ckpt, int32_t ckpt_every, int32_t variant, int32_t flags,
                 void *workspace, size_t workspace_bytes, void *stream);

/* Size of the device array behind sdtw_forward_noalloc (16 MiB per GPU). */
#define SDTW_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)

/*
 * sdtw_forward for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, validation, results and status codes as sdtw_forward,
 * without the workspace: the call uses a fixed device array of
 * SDTW_NOALLOC_SCRATCH_BYTES inside the library instead, and allocates and
 * frees nothing.  Each GPU the library runs on holds its own array until the
 * process ends.
 *
 *   - A batch whose sdtw_forward_workspace_bytes(..., flags, variant)
 *     exceeds SDTW_NOALLOC_SCRATCH_BYTES is rejected with SDTW_ERR_WORKSPACE
 *     before anything is enqueued.  That covers any batch of up to about a
 *     million queries that fit in one row pass of the tile, plus
 *     SDTW_NOALLOC_SCRATCH_BYTES / (4 * ref_len) row-buffer slots for
 *     longer queries (sdtw_forward_workspace_bytes describes the slots).
 *   - The first call on a device looks the array's device address up once
 *     (hipGetSymbolAddress, with that device current; SDTW_ERR_HIP if that
 *     fails); make that first call outside a graph capture.
 *   - All calls on one GPU share that GPU's array, which keeps the last
 *     call's contents (nothing in it needs to start at zero: the persistent
 *     form's work counter is reset by a kernel of the same call).  Calls
 *     that overlap in time on one GPU -- on different streams, or from
 *     different host threads -- race and give undefined results; serialise
 *     them, for example on one stream.
 */
SDTW_API int sdtw_forward_noalloc(const float *queries, const int32_t *h_query_lens,
                                  const int32_t *query_lens, int32_t batch,
                                  const float *reference, int64_t ref_len, int32_t cost_kind,
                                  float *cost, int64_t *end_pos,
                                  float *ckpt, int32_t ckpt_every, int32_t variant,
                                  int32_t flags, void *stream);

/*
 * Bytes of device workspace sdtw_forward_u8 needs: sdtw_forward's (no flags),
 * one byte per query and reference element for the codes, and the codebook.
 * Returns 0 on invalid arguments.
 */
SDTW_API size_t sdtw_forward_u8_workspace_bytes(const int32_t *h_query_lens, int32_t batch,
                                       int64_t ref_len);

/*
 * Forward pass on uint8 codes, the quantisation Section 8 proposes: a
 * codebook built from the reference's values whose bulk is divided evenly
 * over 256 codes, outliers clamped to the end codes.  For z-normalised
 * inputs the bulk is taken as the values within 4 standard deviations of the
 * mean:
 *   lo = max(min(reference), -4),  hi = min(max(reference), 4),
 *   code(x) = clamp(rint((x - lo) * 255 / (hi - lo)), 0, 255)
 * in binary64, round half to even (every code 0 when hi <= lo).  The DP of
 * sdtw_forward then runs in binary32 on the codes taken as numbers 0..255
 * with the local cost (a - b)^2 (exact: at most 65025), so cost is the
 * binary32 DP of the codes -- exact integers while the sums stay below 2^24
 * -- and cost * step^2, step = (hi - lo) / 255, approximates the
 * squared-cost sDTW of the original values.
 *
 *   queries, h_query_lens, query_lens, batch, reference, ref_len, variant,
 *                stream: as for sdtw_forward
 *   cost         device float32 [batch]: minimum of the last row, in units
 *                of step^2 (output)
 *   end_pos      device int64 [batch], 0-based, first minimiser (output)
 *   codebook     device float32 [2]: lo, hi (output)
 *   workspace    device, >= sdtw_forward_u8_workspace_bytes(...) bytes,
 *                256-byte aligned
 */
SDTW_API int sdtw_forward_u8(const float *queries, const int32_t *h_query_lens,
                    const int32_t *query_lens, int32_t batch,
                    const float *reference, int64_t ref_len,
                    float *cost, int64_t *end_pos, float *codebook,
                    int32_t variant, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Forward pass with early pruning, the cost rule Section 8 proposes: after
 * the subtraction t = q_i - r_j, a pair with |t| > prune_tau is taken to be
 * unable to lie on the warp path and costs +inf (no multiplication);
 * otherwise the cost is t*t, as for SDTW_COST_SQUARED.  Everything else is
 * sdtw_forward's: the same DP, outputs, variants and workspace
 * (sdtw_forward_workspace_bytes with the same flags and variant).  The result is an
 * approximation of the squared-cost sDTW: cost[b] >= the exact cost, equal
 * whenever some optimal path has every |t| <= prune_tau (always for
 * prune_tau = +inf); a query with no such path gets +inf and end_pos 0.
 *
 *   prune_tau  any float32 but NaN (NaN: SDTW_ERR_INVALID_ARG); a negative
 *              value prunes every pair
 *   flags      0 or SDTW_F_PERSISTENT (checkpoints: SDTW_ERR_INVALID_ARG)
 *   other arguments as for sdtw_forward
 */
SDTW_API int sdtw_forward_pruned(const float *queries, const int32_t *h_query_lens,
                        const int32_t *query_lens, int32_t batch,
                        const float *reference, int64_t ref_len, float prune_tau,
                        float *cost, int64_t *end_pos, int32_t variant, int32_t flags,
                        void *workspace, size_t workspace_bytes, void *stream);

/*
 * Bytes of device workspace sdtw_backward needs: per-query reference
 * partials (batch x ref_len floats), per-row path bounds, and 2-bit direction
 * codes for the blocks recomputed at once (up to 8 blocks of ckpt_every
 * columns per query, fewer when that would exceed 1 GiB, at least one).
 * Returns 0 on invalid arguments or when a query is longer than 8,192 rows.
 */
SDTW_API size_t sdtw_backward_workspace_bytes(const int32_t *h_query_lens, int32_t batch,
                                     int64_t ref_len, int32_t ckpt_every);

/*
 * Backward pass: gradient of L = sum_b grad_cost[b] * cost_b along each
 * query's optimal warp path, found by walking back (Section 2) from
 * (N, end_pos + 1) to row 1; on ties the walk prefers the diagonal, then the
 * cell above, then the cell to the left.  DP blocks of ckpt_every columns are
 * recomputed from the checkpoints stored by sdtw_forward (same queries,
 * reference, cost kind and ckpt_every, with SDTW_F_CHECKPOINT).  Queries may
 * be at most 8,192 rows long (SDTW_ERR_UNSUPPORTED otherwise).
 *
 * For every path cell (i,j) of query b, term = grad_cost[b] * c'(q_i - r_j)
 * with c'(t) = 2t (squared) or sign(t), sign(0) = 0 (absolute):
 *   grad_queries[offset(b) + i - 1] = sum of term over the path cells of row i,
 *       added in walk order starting from +0;
 *   grad_reference[j - 1] = sum over queries b (increasing b) whose path
 *       touches column j of that query's partial, where the partial is the sum
 *       of -term over the path cells of column j in walk order; +0 for columns
 *       no path touches.
 *
 *   grad_cost       device float32 [batch]
 *   cost            device float32 [batch], as returned by sdtw_forward
 *   end_pos         device int64 [batch], as returned by sdtw_forward
 *   ckpt            device float32, as filled by sdtw_forward (may be NULL
 *                   when sdtw_checkpoint_floats(...) is 0)
 *   grad_queries    device float32, packed like queries (output)
 *   grad_reference  device float32 [ref_len] (output)
 *   workspace       device, >= sdtw_backward_workspace_bytes(...) bytes,
 *                   256-byte aligned
 *   stream          hipStream_t or NULL
 */
SDTW_API int sdtw_backward(const float *queries, const int32_t *h_query_lens,
                  const int32_t *query_lens, int32_t batch,
                  const float *reference, int64_t ref_len, int32_t cost_kind,
                  const float *grad_cost, const float *cost, const int64_t *end_pos,
                  const float *ckpt, int32_t ckpt_every,
                  float *grad_queries, float *grad_reference,
                  void *workspace, size_t workspace_bytes, void *stream);

/*
 * sDTW in binary16, the paper's own precision (Section 5.2 converts queries
 * and reference to half precision and computes on packed pairs; Section 8).
 * Same operation and outputs as sdtw_forward, with every input and every
 * operation (t = q - r, t*t or |t|, min + c) rounded to nearest-even
 * binary16, subnormals kept; values past 65504 become +inf.  cost holds the
 * binary16 result exactly as a float32.  Queries are processed in pairs
 * (2i, 2i+1), one per half of each packed value, so each pair must have
 * equal lengths (else SDTW_ERR_UNSUPPORTED); an odd batch's last query runs
 * alone.  variant: as for sdtw_forward (-1 = library choice); no
 * checkpoints, no persistent form.  workspace:
 * sdtw_forward_f16_workspace_bytes(...) bytes, 256-byte aligned.
 */
SDTW_API size_t sdtw_forward_f16_workspace_bytes(const int32_t *h_query_lens, int32_t batch,
                                                 int64_t ref_len);

SDTW_API int sdtw_forward_f16(const float *queries, const int32_t *h_query_lens,
                              const int32_t *query_lens, int32_t batch,
                              const float *reference, int64_t ref_len, int32_t cost_kind,
                              float *cost, int64_t *end_pos, int32_t variant,
                              void *workspace, size_t workspace_bytes, void *stream);

/*
 * Alignment path of every query (paper: Section 2, the walk back from the
 * minimum of the last row that recovers the optimal warping path), from the
 * outputs of an sdtw_forward call made with SDTW_F_CHECKPOINT.  The walk
 * starts at (N, end_pos), steps to the smallest of the diagonal, upper and
 * left neighbours (ties: diagonal, then up, then left) and stops on row 1.
 * Query element i (row i+1, packed index off_b + i) is matched to reference
 * elements path_lo[off_b + i] .. path_hi[off_b + i] (0-based, inclusive);
 * row ranges are contiguous and consecutive rows touch (path_hi of row i is
 * path_lo of row i+1 or one less).  start_pos[b] = path_lo of query b's
 * first element, so the matched subsequence is reference[start_pos ..
 * end_pos].
 *
 *   cost, end_pos         the forward's outputs for the same inputs
 *   ckpt, ckpt_every      the forward's checkpoint columns and interval
 *   start_pos             int64 [batch]
 *   path_lo, path_hi      int32, packed like queries
 *   workspace             sdtw_align_workspace_bytes(...) bytes, 256-byte
 *                         aligned
 *
 * Same limits and status codes as sdtw_backward (queries of at most 8,192
 * rows, ckpt_every a positive multiple of 16).
 */
SDTW_API size_t sdtw_align_workspace_bytes(const int32_t *h_query_lens, int32_t batch,
                                           int64_t ref_len, int32_t ckpt_every);

SDTW_API int sdtw_align(const float *queries, const int32_t *h_query_lens,
                        const int32_t *query_lens, int32_t batch,
                        const float *reference, int64_t ref_len, int32_t cost_kind,
                        const float *cost, const int64_t *end_pos,
                        const float *ckpt, int32_t ckpt_every,
                        int64_t *start_pos, int32_t *path_lo, int32_t *path_hi,
                        void *workspace, size_t workspace_bytes, void *stream);

/*
 * Batch z-normalisation, the step that prepares queries and reference
 * (paper: Section 5.1, "Normalizer implementation", standardisation equation):
 * every series of a packed batch becomes
 *
 *     z_k = (x_k - mean) / S,   mean = (1/n) sum x_k,
 *     S = sqrt((1/n) sum (x_k - mean)^2)   (population standard deviation),
 *
 * with mean and S in binary64, z = (x_k - mean) * (1/S) in binary64 and
 * rounded once to binary32.  A constant series (S = 0) maps to zeros (the
 * paper leaves it open).  Chunk sums are reduced in a fixed order, so the
 * result does not depend on scheduling; it is within one binary32 ulp of the
 * definition evaluated in binary64 in any other order.
 *
 *   x             packed float32 series [sum h_lens] (packed like queries)
 *   h_lens/lens   host / device int32 [batch] series lengths, each >= 1
 *   z             float32 output packed like x; either equal to x (in place)
 *                 or not overlapping it
 *   workspace     sdtw_znorm_workspace_bytes(h_lens, batch) bytes, 256-byte
 *                 aligned; contents on return are unspecified
 *
 * Returns SDTW_OK, SDTW_ERR_INVALID_ARG (null pointer, batch < 1, a length
 * < 1, misaligned workspace), SDTW_ERR_WORKSPACE or SDTW_ERR_HIP.
 */
SDTW_API size_t sdtw_znorm_workspace_bytes(const int32_t *h_lens, int32_t batch);

SDTW_API int sdtw_znorm(const float *x, const int32_t *h_lens, const int32_t *lens,
                        int32_t batch, float *z, void *workspace, size_t workspace_bytes,
                        void *stream);

/* Number of compiled forward tile variants. */
SDTW_API int32_t sdtw_variant_count(void);

/*
 * Describe variant v: query rows held per lane, reference columns per step,
 * wavefronts per query, steps between workgroup barriers, and how a lane's
 * bottom row reaches the next lane (1: through LDS, 0: DPP lane shift).  Any
 * output pointer may be NULL.  Returns SDTW_OK or SDTW_ERR_UNSUPPORTED.
 */
SDTW_API int sdtw_variant_info(int32_t v, int32_t *rows_per_lane, int32_t *tile_cols,
                               int32_t *waves, int32_t *steps_per_barrier,
                               int32_t *lane_exchange);

/* Variant the library picks for this batch when variant = -1. */
SDTW_API int32_t sdtw_default_variant(const int32_t *h_query_lens, int32_t batch,
                             int64_t ref_len, int32_t flags);

/* Static description of a status code (never NULL). */
SDTW_API const char *sdtw_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* SDTW_H */
