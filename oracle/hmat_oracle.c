/*
 * Oracle for the H-matrix-vector product -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this file's library. The GPU library never links, includes or calls it, and
 * the two share no source.
 *
 * What it computes (Sec. 2, Eq. (2.4) "hmat-vec-add"): starting from y = 0,
 * every block of the H-matrix adds its product to the target rows,
 *     dense block (t,s):    y_t += D_ts x_s
 *     low-rank block (t,s): y_t += U_ts (V_ts^T x_s)
 * and the GEMV form of the remark that closes Sec. 4.1 returns
 *     y_out = alpha * y + beta * y_in      (y_in is not read when beta == 0).
 * The method reaches exactly this result up to the order of the additions, so
 * the oracle is this definition written out. All arithmetic is FP64; the FP32
 * factors are promoted exactly.
 *
 * Factor layout (one pool of floats): a dense block is |t| x |s| column-major
 * at pool + off_a[b]; a low-rank block has U (|t| x r) at pool + off_a[b] and
 * V (|s| x r) at pool + off_b[b], both column-major with leading dimension equal
 * to their row count.
 *
 * Threading changes only which thread adds which rows: pass 1 forms
 * w_b = V_b^T x_s for every low-rank block (one block per iteration); pass 2
 * gives each thread a disjoint range of output rows, and the thread adds, for
 * every block, the rows of D_ts x_s or U_ts w_b that fall in its range.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

int hmat_oracle_matvec(int64_t n, int64_t num_blocks,
                       const int64_t *row_begin, const int64_t *row_end,
                       const int64_t *col_begin, const int64_t *col_end,
                       const int32_t *rank, const float *pool,
                       const int64_t *off_a, const int64_t *off_b,
                       int32_t nrhs, double alpha, const double *x, int64_t ldx,
                       double beta, double *y, int64_t ldy,
                       int64_t row_lo, int64_t row_hi, int32_t nthreads)
{
    if (n <= 0 || num_blocks < 0 || nrhs < 1 || ldx < n || ldy < n)
        return -1;
    if (!row_begin || !row_end || !col_begin || !col_end || !rank || !pool || !off_a ||
        !off_b || !x || !y)
        return -1;
    if (row_lo < 0 || row_hi > n || row_lo >= row_hi)
        return -1;
    if (nthreads < 1)
        nthreads = omp_get_max_threads();

    /* w holds V_b^T x_s for every low-rank block, one column at a time. */
    int64_t *w_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(num_blocks + 1));
    if (!w_off)
        return -2;
    w_off[0] = 0;
    for (int64_t b = 0; b < num_blocks; ++b)
        w_off[b + 1] = w_off[b] + (rank[b] > 0 ? rank[b] : 0);
    double *w = (double *)malloc(sizeof(double) * (size_t)(w_off[num_blocks] + 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(row_hi - row_lo));
    if (!w || !acc) {
        free(w_off);
        free(w);
        free(acc);
        return -2;
    }

    for (int32_t c = 0; c < nrhs; ++c) {
        const double *xc = x + (int64_t)c * ldx;
        double *yc = y + (int64_t)c * ldy;

        /* Pass 1: w_b = V_b^T x_s (Eq. (2.4), inner product of the low-rank term). */
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
        for (int64_t b = 0; b < num_blocks; ++b) {
            if (rank[b] <= 0)
                continue;
            if (row_end[b] <= row_lo || row_begin[b] >= row_hi)
                continue;
            const int64_t ns = col_end[b] - col_begin[b];
            const float *v = pool + off_b[b];
            for (int32_t k = 0; k < rank[b]; ++k) {
                double s = 0.0;
                for (int64_t i = 0; i < ns; ++i)
                    s += (double)v[(int64_t)k * ns + i] * xc[col_begin[b] + i];
                w[w_off[b] + k] = s;
            }
        }

        /* Pass 2: y_t += D_ts x_s and y_t += U_ts w_b, rows split among threads. */
#pragma omp parallel num_threads(nthreads)
        {
            const int nt = omp_get_num_threads();
            const int me = omp_get_thread_num();
            const int64_t span = row_hi - row_lo;
            const int64_t lo = row_lo + span * me / nt;
            const int64_t hi = row_lo + span * (me + 1) / nt;
            for (int64_t i = lo; i < hi; ++i)
                acc[i - row_lo] = 0.0;
            for (int64_t b = 0; b < num_blocks && lo < hi; ++b) {
                const int64_t r0 = row_begin[b] > lo ? row_begin[b] : lo;
                const int64_t r1 = row_end[b] < hi ? row_end[b] : hi;
                if (r0 >= r1)
                    continue;
                const int64_t mt = row_end[b] - row_begin[b];
                if (rank[b] == 0) {
                    const int64_t ns = col_end[b] - col_begin[b];
                    const float *d = pool + off_a[b];
                    for (int64_t j = 0; j < ns; ++j) {
                        const double xj = xc[col_begin[b] + j];
                        const float *dj = d + j * mt;
                        for (int64_t i = r0; i < r1; ++i)
                            acc[i - row_lo] += (double)dj[i - row_begin[b]] * xj;
                    }
                } else {
                    const float *u = pool + off_a[b];
                    for (int32_t k = 0; k < rank[b]; ++k) {
                        const double wk = w[w_off[b] + k];
                        const float *uk = u + (int64_t)k * mt;
                        for (int64_t i = r0; i < r1; ++i)
                            acc[i - row_lo] += (double)uk[i - row_begin[b]] * wk;
                    }
                }
            }
            for (int64_t i = lo; i < hi; ++i)
                yc[i] = (beta == 0.0) ? alpha * acc[i - row_lo]
                                      : alpha * acc[i - row_lo] + beta * yc[i];
        }
    }
    free(w_off);
    free(w);
    free(acc);
    return 0;
}

int hmat_oracle_max_threads(void) { return omp_get_max_threads(); }
