/*
 * sdtw_oracle.c -- CPU oracle for subsequence dynamic time warping (sDTW).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU path computes.  Only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or helper with the HIP library, and the HIP library never
 * calls it.
 *
 * What is computed (paper: Section 2, Eq. (1) and the paragraph after it):
 *
 *   D(i,j) = min{ D(i-1,j), D(i,j-1), D(i-1,j-1) } + d(X_i, Y_j)
 *
 * with X the query (rows i = 1..N) and Y the reference (columns j = 1..M).
 * The subsequence variant (Section 2: the query fits the best segment of the
 * reference) is obtained by the initialisation
 *
 *   D(0,j) = 0      for j = 0..M       (free start anywhere in the reference)
 *   D(i,0) = +inf   for i = 1..N
 *
 * and the result is the minimum of the last row, cost = min_j D(N,j), with
 * end_pos = (smallest j attaining it) - 1, i.e. the 0-based index of the
 * reference element matched to the last query element.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - d is the squared difference (Section 8 mentions a subtraction followed
 *     by a multiplication) or the absolute difference; kind 0 / kind 1.
 *     Kind 2 is Section 8's early pruning: the squared difference, but +inf
 *     when |q - r| > tau (strictly), decided before the multiplication.
 *   - FP32 arithmetic is t = q - r, c = t*t (or |t|), D = m + c, each rounded
 *     to nearest-even, with no fused multiply-add (build with
 *     -ffp-contract=off) and no flush of subnormals.
 *   - min{} is exact and is written as plain comparisons.
 *   - the walk-back (Section 2: from the minimum of the last row, follow the
 *     neighbour with the smallest accumulated cost) takes, on ties, the
 *     diagonal first, then the cell above, then the cell to the left.
 *
 * The FP64 twin widens the FP32 inputs exactly and does all arithmetic in
 * binary64; it is the accuracy reference, not a bit-exact target.  The
 * binary16 twin (the paper's own precision, Section 5.2) rounds every input
 * and every operation result to binary16; see oracle_round_f16.
 *
 * Parity pins for every function here live in tests/test_oracle_*.py:
 * brute-force enumeration of all warp paths (in binary32 and in binary16), a
 * hand-worked DP matrix, the N = 1 closed form, exact-excerpt zeros, path
 * upper bounds, FP32/FP64 agreement within the rounding-error bound, finite
 * differences of the FP64 cost for the gradient, and NumPy's float16
 * conversion for the binary16 rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORACLE_SQUARED = 0, ORACLE_ABSOLUTE = 1, ORACLE_PRUNED = 2 };

/* ------------------------------------------------------------------ */
/* Local cost d(X_i, Y_j) and the exact three-way minimum.             */
/* ------------------------------------------------------------------ */

static float local_cost_f32(float q, float r, int kind, float tau)
{
    float t = q - r;
    if (kind == ORACLE_SQUARED) {
        float c = t * t;
        return c;
    }
    if (kind == ORACLE_PRUNED) {
        /* Early pruning (Section 8): decided on the difference, before any
         * multiplication; a pair farther apart than tau cannot be on the
         * path and costs +inf. */
        if (fabsf(t) > tau) return INFINITY;
        float c = t * t;
        return c;
    }
    return fabsf(t);
}

static double local_cost_f64(double q, double r, int kind)
{
    double t = q - r;
    if (kind == ORACLE_SQUARED) {
        double c = t * t;
        return c;
    }
    return fabs(t);
}

static float min3_f32(float a, float b, float c)
{
    float m = a;
    if (b < m) m = b;
    if (c < m) m = c;
    return m;
}

static double min3_f64(double a, double b, double c)
{
    double m = a;
    if (b < m) m = b;
    if (c < m) m = c;
    return m;
}

/* ------------------------------------------------------------------ */
/* One query, two rolling DP rows of M+1 entries (column 0 is the      */
/* +inf boundary).                                                     */
/* ------------------------------------------------------------------ */

static void sdtw_one_f32(const float *q, int64_t n, const float *r, int64_t m,
                         int kind, float tau, float *prev, float *cur,
                         float *cost, int64_t *end_pos)
{
    for (int64_t j = 0; j <= m; ++j) prev[j] = 0.0f;       /* row 0 */
    for (int64_t i = 1; i <= n; ++i) {
        cur[0] = INFINITY;                                  /* column 0 */
        float qi = q[i - 1];
        for (int64_t j = 1; j <= m; ++j) {
            float c = local_cost_f32(qi, r[j - 1], kind, tau);
            float mn = min3_f32(prev[j], cur[j - 1], prev[j - 1]);
            cur[j] = mn + c;
        }
        float *t = prev; prev = cur; cur = t;
    }
    /* prev now holds row N */
    float best = prev[1];
    int64_t arg = 1;
    for (int64_t j = 2; j <= m; ++j) {
        if (prev[j] < best) { best = prev[j]; arg = j; }
    }
    *cost = best;
    *end_pos = arg - 1;
}

static void sdtw_one_f64(const float *q, int64_t n, const float *r, int64_t m,
                         int kind, double *prev, double *cur,
                         double *cost, int64_t *end_pos)
{
    for (int64_t j = 0; j <= m; ++j) prev[j] = 0.0;
    for (int64_t i = 1; i <= n; ++i) {
        cur[0] = INFINITY;
        double qi = (double)q[i - 1];
        for (int64_t j = 1; j <= m; ++j) {
            double c = local_cost_f64(qi, (double)r[j - 1], kind);
            double mn = min3_f64(prev[j], cur[j - 1], prev[j - 1]);
            cur[j] = mn + c;
        }
        double *t = prev; prev = cur; cur = t;
    }
    double best = prev[1];
    int64_t arg = 1;
    for (int64_t j = 2; j <= m; ++j) {
        if (prev[j] < best) { best = prev[j]; arg = j; }
    }
    *cost = best;
    *end_pos = arg - 1;
}

/* ------------------------------------------------------------------ */
/* Binary16 (the paper's own precision, Section 5.2 and Section 8):     */
/* every input and every operation result is rounded to the nearest     */
/* binary16 value, ties to even.  Values are carried in doubles: the    */
/* difference, product or sum of two binary16 numbers is exact in       */
/* binary64 (at most 41 significant bits), so one rounding per          */
/* operation gives the correctly rounded binary16 result.               */
/* ------------------------------------------------------------------ */

/* Nearest binary16 value of x (ties to even), as a double.  binary16 has
 * an 11-bit significand, normal exponents -14..15 and subnormal spacing
 * 2^-24; magnitudes from 65520 (the midpoint between the largest finite
 * value 65504 and 2^16, which rounds to the even side) up overflow to inf. */
double oracle_round_f16(double x)
{
    if (x != x || x == 0.0 || isinf(x)) return x;
    int e;
    frexp(fabs(x), &e);                  /* |x| = f * 2^e, f in [0.5, 1) */
    int ex = e - 1;                      /* |x| in [2^ex, 2^(ex+1)) */
    if (ex < -14) ex = -14;              /* subnormal range: fixed spacing */
    double quantum = ldexp(1.0, ex - 10);
    double r = nearbyint(x / quantum) * quantum;   /* exact scaling, RNE */
    if (fabs(r) > 65504.0) return copysign(INFINITY, x);
    return r;
}

static double local_cost_f16(double q, double r, int kind)
{
    double t = oracle_round_f16(q - r);
    if (kind == ORACLE_SQUARED) return oracle_round_f16(t * t);
    return fabs(t);
}

/* One query in binary16 arithmetic (values held as doubles). */
static void sdtw_one_f16(const float *q, int64_t n, const float *r, int64_t m,
                         int kind, double *prev, double *cur,
                         float *cost, int64_t *end_pos)
{
    for (int64_t j = 0; j <= m; ++j) prev[j] = 0.0;
    for (int64_t i = 1; i <= n; ++i) {
        cur[0] = INFINITY;
        double qi = oracle_round_f16((double)q[i - 1]);
        for (int64_t j = 1; j <= m; ++j) {
            double c = local_cost_f16(qi, oracle_round_f16((double)r[j - 1]), kind);
            double mn = min3_f64(prev[j], cur[j - 1], prev[j - 1]);
            cur[j] = oracle_round_f16(mn + c);
        }
        double *t = prev; prev = cur; cur = t;
    }
    double best = prev[1];
    int64_t arg = 1;
    for (int64_t j = 2; j <= m; ++j) {
        if (prev[j] < best) { best = prev[j]; arg = j; }
    }
    *cost = (float)best;                 /* a binary16 value: exact in binary32 */
    *end_pos = arg - 1;
}

/* Query b of a packed batch starts at the sum of the lengths before it. */
static int64_t *make_offsets(const int32_t *lens, int32_t batch)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)batch + 1));
    if (!off) return NULL;
    off[0] = 0;
    for (int32_t b = 0; b < batch; ++b) off[b + 1] = off[b] + lens[b];
    return off;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Number of threads an OpenMP parallel region will use (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Batched FP32 sDTW.  queries: packed, query b has lens[b] floats.
 * Returns 0 on success, -1 on a bad argument or allocation failure.
 */
static int sdtw_batch_f32(const float *queries, const int32_t *lens, int32_t batch,
                          const float *ref, int64_t ref_len, int kind, float tau,
                          float *cost, int64_t *end_pos, int nthreads)
{
    for (int32_t b = 0; b < batch; ++b) if (lens[b] < 1) return -1;
    int64_t *off = make_offsets(lens, batch);
    if (!off) return -1;
    int failed = 0;
    set_threads(nthreads);
#pragma omp parallel
    {
        float *prev = (float *)malloc(sizeof(float) * (size_t)(ref_len + 1));
        float *cur = (float *)malloc(sizeof(float) * (size_t)(ref_len + 1));
        if (!prev || !cur) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int32_t b = 0; b < batch; ++b)
                sdtw_one_f32(queries + off[b], lens[b], ref, ref_len, kind, tau,
                             prev, cur, &cost[b], &end_pos[b]);
        }
        free(prev);
        free(cur);
    }
    free(off);
    return failed ? -1 : 0;
}

/*
 * Batched FP32 sDTW.  queries: packed, query b has lens[b] floats.
 * Returns 0 on success, -1 on a bad argument or allocation failure.
 */
int oracle_sdtw_f32(const float *queries, const int32_t *lens, int32_t batch,
                    const float *ref, int64_t ref_len, int kind,
                    float *cost, int64_t *end_pos, int nthreads)
{
    if (batch < 1 || ref_len < 1 || (kind != 0 && kind != 1)) return -1;
    return sdtw_batch_f32(queries, lens, batch, ref, ref_len, kind, INFINITY,
                          cost, end_pos, nthreads);
}

/*
 * Batched FP32 sDTW with early pruning (Section 8): the squared cost, except
 * that a pair with |q - r| > tau costs +inf.  tau must not be NaN.
 */
int oracle_sdtw_pruned_f32(const float *queries, const int32_t *lens, int32_t batch,
                           const float *ref, int64_t ref_len, float tau,
                           float *cost, int64_t *end_pos, int nthreads)
{
    if (batch < 1 || ref_len < 1 || isnan(tau)) return -1;
    return sdtw_batch_f32(queries, lens, batch, ref, ref_len, ORACLE_PRUNED, tau,
                          cost, end_pos, nthreads);
}

/* Batched FP64 twin of oracle_sdtw_f32 (inputs widened exactly). */
int oracle_sdtw_f64(const float *queries, const int32_t *lens, int32_t batch,
                    const float *ref, int64_t ref_len, int kind,
                    double *cost, int64_t *end_pos, int nthreads)
{
    if (batch < 1 || ref_len < 1 || (kind != 0 && kind != 1)) return -1;
    for (int32_t b = 0; b < batch; ++b) if (lens[b] < 1) return -1;
    int64_t *off = make_offsets(lens, batch);
    if (!off) return -1;
    int failed = 0;
    set_threads(nthreads);
#pragma omp parallel
    {
        double *prev = (double *)malloc(sizeof(double) * (size_t)(ref_len + 1));
        double *cur = (double *)malloc(sizeof(double) * (size_t)(ref_len + 1));
        if (!prev || !cur) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int32_t b = 0; b < batch; ++b)
                sdtw_one_f64(queries + off[b], lens[b], ref, ref_len, kind,
                             prev, cur, &cost[b], &end_pos[b]);
        }
        free(prev);
        free(cur);
    }
    free(off);
    return failed ? -1 : 0;
}

/* Batched binary16 sDTW (inputs rounded to binary16; costs returned as the
 * binary32 values of the binary16 results). */
int oracle_sdtw_f16(const float *queries, const int32_t *lens, int32_t batch,
                    const float *ref, int64_t ref_len, int kind,
                    float *cost, int64_t *end_pos, int nthreads)
{
    if (batch < 1 || ref_len < 1 || (kind != 0 && kind != 1)) return -1;
    for (int32_t b = 0; b < batch; ++b) if (lens[b] < 1) return -1;
    int64_t *off = make_offsets(lens, batch);
    if (!off) return -1;
    int failed = 0;
    set_threads(nthreads);
#pragma omp parallel
    {
        double *prev = (double *)malloc(sizeof(double) * (size_t)(ref_len + 1));
        double *cur = (double *)malloc(sizeof(double) * (size_t)(ref_len + 1));
        if (!prev || !cur) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int32_t b = 0; b < batch; ++b)
                sdtw_one_f16(queries + off[b], lens[b], ref, ref_len, kind,
                             prev, cur, &cost[b], &end_pos[b]);
        }
        free(prev);
        free(cur);
    }
    free(off);
    return failed ? -1 : 0;
}

/*
 * Last DP row of one query in FP32: out[j-1] = D(N, j) for j = 1..M.
 * Used by tests that need the whole row (for example the end-position
 * tie-break or the monotonicity pins).
 */
int oracle_sdtw_last_row_f32(const float *q, int32_t n, const float *ref,
                             int64_t ref_len, int kind, float *out)
{
    if (n < 1 || ref_len < 1 || (kind != 0 && kind != 1)) return -1;
    float *prev = (float *)malloc(sizeof(float) * (size_t)(ref_len + 1));
    float *cur = (float *)malloc(sizeof(float) * (size_t)(ref_len + 1));
    if (!prev || !cur) { free(prev); free(cur); return -1; }
    for (int64_t j = 0; j <= ref_len; ++j) prev[j] = 0.0f;
    for (int64_t i = 1; i <= n; ++i) {
        cur[0] = INFINITY;
        for (int64_t j = 1; j <= ref_len; ++j) {
            float c = local_cost_f32(q[i - 1], ref[j - 1], kind, INFINITY);
            cur[j] = min3_f32(prev[j], cur[j - 1], prev[j - 1]) + c;
        }
        float *t = prev; prev = cur; cur = t;
    }
    memcpy(out, prev + 1, sizeof(float) * (size_t)ref_len);
    free(prev);
    free(cur);
    return 0;
}

/*
 * Global (corner-to-corner) DTW in FP32, the textbook alignment of Section 2:
 * D(0,0) = 0, D(0,j>0) = D(i>0,0) = +inf, result D(N,M).  The tests use it
 * as an upper bound on the subsequence cost; it is pinned on its own by a
 * brute-force enumeration of every corner-to-corner warp path (bit for bit
 * in binary32) and by a hand-worked table of the 3 x 6 example.
 */
int oracle_dtw_f32(const float *q, int32_t n, const float *ref,
                   int64_t ref_len, int kind, float *out)
{
    if (n < 1 || ref_len < 1 || (kind != 0 && kind != 1)) return -1;
    float *prev = (float *)malloc(sizeof(float) * (size_t)(ref_len + 1));
    float *cur = (float *)malloc(sizeof(float) * (size_t)(ref_len + 1));
    if (!prev || !cur) { free(prev); free(cur); return -1; }
    prev[0] = 0.0f;
    for (int64_t j = 1; j <= ref_len; ++j) prev[j] = INFINITY;
    for (int64_t i = 1; i <= n; ++i) {
        cur[0] = INFINITY;
        for (int64_t j = 1; j <= ref_len; ++j) {
            float c = local_cost_f32(q[i - 1], ref[j - 1], kind, INFINITY);
            cur[j] = min3_f32(prev[j], cur[j - 1], prev[j - 1]) + c;
        }
        float *t = prev; prev = cur; cur = t;
    }
    *out = prev[ref_len];
    free(prev);
    free(cur);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Gradient by walk-back over the full FP32 matrix.                    */
/* ------------------------------------------------------------------ */

/*
 * Derivative of the local cost with respect to the query value, at
 * t = q - r: squared -> 2t, absolute -> sign(t) with sign(0) = 0.
 * The derivative with respect to the reference value is its negation.
 */
static float dcost_dq_f32(float q, float r, int kind)
{
    float t = q - r;
    if (kind == ORACLE_SQUARED) return 2.0f * t;
    if (t > 0.0f) return 1.0f;
    if (t < 0.0f) return -1.0f;
    return 0.0f;
}

/*
 * Fill the full (n+1) x (m+1) FP32 matrix of one query (row-major, row
 * stride m+1) and return the walk-back path from (n, end+1) to row 1.
 * path_i / path_j receive 1-based cell coordinates in walk order (from the
 * end cell back to the start cell); *path_len the number of cells.
 */
static void sdtw_full_and_walk(const float *q, int64_t n, const float *r,
                               int64_t m, int kind, float *D,
                               int64_t *path_i, int64_t *path_j,
                               int64_t *path_len, float *cost, int64_t *end_pos)
{
    const int64_t s = m + 1;
    for (int64_t j = 0; j <= m; ++j) D[j] = 0.0f;
    for (int64_t i = 1; i <= n; ++i) {
        float *row = D + i * s;
        const float *up = D + (i - 1) * s;
        row[0] = INFINITY;
        for (int64_t j = 1; j <= m; ++j) {
            float c = local_cost_f32(q[i - 1], r[j - 1], kind, INFINITY);
            row[j] = min3_f32(up[j], row[j - 1], up[j - 1]) + c;
        }
    }
    const float *last = D + n * s;
    float best = last[1];
    int64_t jb = 1;
    for (int64_t j = 2; j <= m; ++j)
        if (last[j] < best) { best = last[j]; jb = j; }
    *cost = best;
    *end_pos = jb - 1;

    /* Walk back: ties go to the diagonal, then up, then left. */
    int64_t i = n, j = jb, k = 0;
    for (;;) {
        path_i[k] = i;
        path_j[k] = j;
        ++k;
        if (i == 1) break;
        float vd = D[(i - 1) * s + (j - 1)];
        float vu = D[(i - 1) * s + j];
        float vl = D[i * s + (j - 1)];
        int64_t ni = i - 1, nj = j - 1;
        float bv = vd;
        if (vu < bv) { bv = vu; ni = i - 1; nj = j; }
        if (vl < bv) { bv = vl; ni = i; nj = j - 1; }
        i = ni;
        j = nj;
    }
    *path_len = k;
}

/*
 * FP32 cost, end position and gradient of L = sum_b grad_cost[b] * cost_b.
 *
 *   grad_queries (packed like queries): for every path cell (i,j) of query b,
 *       term = grad_cost[b] * dd(q_i, r_j), accumulated into row i in walk
 *       order (from the end cell back to the start cell), starting at +0.
 *   grad_ref[j]: per query, the terms -term of the path cells in column j
 *       are summed in walk order into a partial; the partials of the queries
 *       whose path touches column j are then added in increasing b order,
 *       starting at +0.  Columns touched by no path get +0.
 *
 * path_start (optional, may be NULL): 0-based reference index where each
 * query's path starts (its cell in row 1).
 *
 * Memory: one (N+1)(M+1) float matrix per thread.
 */
int oracle_sdtw_grad_f32(const float *queries, const int32_t *lens,
                         int32_t batch, const float *ref, int64_t ref_len,
                         int kind, const float *grad_cost,
                         float *cost, int64_t *end_pos, int64_t *path_start,
                         float *grad_queries, float *grad_ref, int nthreads)
{
    if (batch < 1 || ref_len < 1 || (kind != 0 && kind != 1)) return -1;
    for (int32_t b = 0; b < batch; ++b) if (lens[b] < 1) return -1;
    int64_t *off = make_offsets(lens, batch);
    if (!off) return -1;
    /* per-query partial of grad_ref over its column range [lo, hi] */
    float **part = (float **)calloc((size_t)batch, sizeof(float *));
    int64_t *lo = (int64_t *)malloc(sizeof(int64_t) * (size_t)batch);
    int64_t *hi = (int64_t *)malloc(sizeof(int64_t) * (size_t)batch);
    if (!part || !lo || !hi) { free(off); free(part); free(lo); free(hi); return -1; }
    int failed = 0;
    set_threads(nthreads);
#pragma omp parallel
    {
        int32_t nmax = 0;
        for (int32_t b = 0; b < batch; ++b) if (lens[b] > nmax) nmax = lens[b];
        size_t cells = (size_t)(nmax + 1) * (size_t)(ref_len + 1);
        float *D = (float *)malloc(sizeof(float) * cells);
        size_t pmax = (size_t)nmax + (size_t)ref_len + 1;
        int64_t *pi = (int64_t *)malloc(sizeof(int64_t) * pmax);
        int64_t *pj = (int64_t *)malloc(sizeof(int64_t) * pmax);
        if (!D || !pi || !pj) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int32_t b = 0; b < batch; ++b) {
                const float *q = queries + off[b];
                int64_t n = lens[b], plen = 0;
                sdtw_full_and_walk(q, n, ref, ref_len, kind, D, pi, pj, &plen,
                                   &cost[b], &end_pos[b]);
                float *gq = grad_queries + off[b];
                for (int64_t i = 0; i < n; ++i) gq[i] = 0.0f;
                int64_t jlo = pj[plen - 1] - 1, jhi = pj[0] - 1;
                float *pr = (float *)malloc(sizeof(float) * (size_t)(jhi - jlo + 1));
                if (!pr) {
#pragma omp atomic write
                    failed = 1;
                    continue;
                }
                for (int64_t j = 0; j <= jhi - jlo; ++j) pr[j] = 0.0f;
                for (int64_t k = 0; k < plen; ++k) {
                    int64_t i0 = pi[k] - 1, j0 = pj[k] - 1;
                    float d = dcost_dq_f32(q[i0], ref[j0], kind);
                    float term = grad_cost[b] * d;
                    gq[i0] = gq[i0] + term;
                    pr[j0 - jlo] = pr[j0 - jlo] + (-term);
                }
                part[b] = pr;
                lo[b] = jlo;
                hi[b] = jhi;
                if (path_start) path_start[b] = jlo;
            }
        }
        free(D);
        free(pi);
        free(pj);
    }
    if (!failed) {
        for (int64_t j = 0; j < ref_len; ++j) grad_ref[j] = 0.0f;
        /* fixed increasing-b order: deterministic */
        for (int32_t b = 0; b < batch; ++b)
            for (int64_t j = lo[b]; j <= hi[b]; ++j)
                grad_ref[j] = grad_ref[j] + part[b][j - lo[b]];
    }
    for (int32_t b = 0; b < batch; ++b) free(part[b]);
    free(part);
    free(lo);
    free(hi);
    free(off);
    return failed ? -1 : 0;
}

/*
 * Walk-back path of one query (FP32), for tests: cells in walk order as
 * 0-based (row, reference index) pairs.  Returns the number of cells, or -1.
 * out_i / out_j must hold n + ref_len entries.
 */
int64_t oracle_sdtw_path_f32(const float *q, int32_t n, const float *ref,
                             int64_t ref_len, int kind,
                             int64_t *out_i, int64_t *out_j)
{
    if (n < 1 || ref_len < 1 || (kind != 0 && kind != 1)) return -1;
    float *D = (float *)malloc(sizeof(float) * (size_t)(n + 1) * (size_t)(ref_len + 1));
    if (!D) return -1;
    int64_t plen = 0, e = 0;
    float c = 0.0f;
    sdtw_full_and_walk(q, n, ref, ref_len, kind, D, out_i, out_j, &plen, &c, &e);
    for (int64_t k = 0; k < plen; ++k) { out_i[k] -= 1; out_j[k] -= 1; }
    free(D);
    return plen;
}

/* ------------------------------------------------------------------ */
/* sDTW on uint8 codes (Section 8's proposed quantisation) in exact     */
/* integer arithmetic, local cost (a - b)^2: the twin that pins the     */
/* binary32 DP of the codes while its sums stay below 2^24.             */
/* ------------------------------------------------------------------ */

static void sdtw_one_codes(const uint8_t *q, int64_t n, const uint8_t *r, int64_t m,
                           int64_t *prev, int64_t *cur, int64_t *cost, int64_t *end_pos)
{
    const int64_t inf = INT64_MAX;                  /* column 0; never added to */
    for (int64_t j = 0; j <= m; ++j) prev[j] = 0;   /* row 0 */
    for (int64_t i = 1; i <= n; ++i) {
        cur[0] = inf;
        for (int64_t j = 1; j <= m; ++j) {
            int64_t t = (int64_t)q[i - 1] - (int64_t)r[j - 1];
            int64_t mn = prev[j];
            if (cur[j - 1] < mn) mn = cur[j - 1];
            if (prev[j - 1] < mn) mn = prev[j - 1];
            cur[j] = mn + t * t;
        }
        int64_t *tmp = prev; prev = cur; cur = tmp;
    }
    int64_t best = prev[1], arg = 1;
    for (int64_t j = 2; j <= m; ++j)
        if (prev[j] < best) { best = prev[j]; arg = j; }
    *cost = best;
    *end_pos = arg - 1;
}

/* Batched sDTW on codes; queries packed like oracle_sdtw_f32's. */
int oracle_sdtw_codes(const uint8_t *queries, const int32_t *lens, int32_t batch,
                      const uint8_t *ref, int64_t ref_len, int64_t *cost, int64_t *end_pos,
                      int nthreads)
{
    if (batch < 1 || ref_len < 1) return -1;
    for (int32_t b = 0; b < batch; ++b) if (lens[b] < 1) return -1;
    int64_t *off = make_offsets(lens, batch);
    if (!off) return -1;
    int failed = 0;
    set_threads(nthreads);
#pragma omp parallel
    {
        int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ref_len + 1));
        int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ref_len + 1));
        if (!prev || !cur) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int32_t b = 0; b < batch; ++b)
                sdtw_one_codes(queries + off[b], lens[b], ref, ref_len, prev, cur,
                               &cost[b], &end_pos[b]);
        }
        free(prev);
        free(cur);
    }
    free(off);
    return failed ? -1 : 0;
}
