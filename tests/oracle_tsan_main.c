/* Runs the OpenMP oracle (oracle/hmat_oracle.c) once over a structure file in
 * the format of tests/sanitize_driver.cpp (magic 1), for a ThreadSanitizer
 * build; prints the result's sum. Used by tests/test_sanitize_cpu.py only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int hmat_oracle_matvec(int64_t n, int64_t num_blocks, const int64_t *row_begin, const int64_t *row_end,
                       const int64_t *col_begin, const int64_t *col_end, const int32_t *rank, const float *pool,
                       const int64_t *off_a, const int64_t *off_b, int32_t nrhs, double alpha, const double *x,
                       int64_t ldx, double beta, double *y, int64_t ldy, int64_t row_lo, int64_t row_hi,
                       int32_t nthreads);

static void rd(FILE *f, void *p, size_t sz, size_t n) {
    if (n && fread(p, sz, n, f) != n) exit(2);
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t magic, nn, nb, d;
    int64_t n;
    rd(f, &magic, 4, 1);
    rd(f, &n, 8, 1);
    rd(f, &nn, 4, 1);
    rd(f, &nb, 4, 1);
    rd(f, &d, 4, 1);
    int32_t *parent = malloc(4 * nn);
    int64_t *begin = malloc(8 * nn), *end = malloc(8 * nn);
    rd(f, parent, 4, nn);
    rd(f, begin, 8, nn);
    rd(f, end, 8, nn);
    int32_t *target = malloc(4 * nb), *source = malloc(4 * nb), *rank = malloc(4 * nb);
    int64_t *off_a = malloc(8 * nb), *off_b = malloc(8 * nb);
    rd(f, target, 4, nb);
    rd(f, source, 4, nb);
    rd(f, rank, 4, nb);
    rd(f, off_a, 8, nb);
    rd(f, off_b, 8, nb);
    int64_t ps;
    rd(f, &ps, 8, 1);
    float *pool = malloc(4 * ps);
    rd(f, pool, 4, ps);
    fclose(f);
    int64_t *rb = malloc(8 * nb), *re = malloc(8 * nb), *cb = malloc(8 * nb), *ce = malloc(8 * nb);
    for (int32_t b = 0; b < nb; ++b) {
        rb[b] = begin[target[b]];
        re[b] = end[target[b]];
        cb[b] = begin[source[b]];
        ce[b] = end[source[b]];
    }
    double *x = malloc(8 * 2 * n), *y = malloc(8 * 2 * n);
    for (int64_t i = 0; i < 2 * n; ++i) x[i] = (double)((i * 7919) % 101) / 101.0 - 0.5;
    const int rc = hmat_oracle_matvec(n, nb, rb, re, cb, ce, rank, pool, off_a, off_b, 2, 1.0, x, n, 0.0, y, n, 0,
                                      n, 4);
    double s = 0.0;
    for (int64_t i = 0; i < 2 * n; ++i) s += y[i];
    printf("rc %d sum %.6e\n", rc, s);
    free(parent); free(begin); free(end); free(target); free(source); free(rank); free(off_a); free(off_b);
    free(pool); free(rb); free(re); free(cb); free(ce); free(x); free(y);
    return rc;
}
