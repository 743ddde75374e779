/* The C oracle (test infrastructure) run under AddressSanitizer and UBSan on
 * small ragged systems: weights, alias table, sampler, slice order, residual,
 * plain / delayed / slice / single-coordinate runs with curves, and replayed
 * rows.  Exit status 0 = every call returned OK and the memory checks held. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t orc_row_weights(int64_t m, const int64_t *row_ptr, const double *val, double *w);
int orc_alias_build(int64_t m, const double *w, uint64_t *thresh, int32_t *alias);
int orc_sample_rows(int64_t m, uint64_t seed, uint32_t stream, const uint64_t *thresh, const int32_t *alias,
                    int64_t ticket0, int64_t count, int32_t *rows_out, uint32_t *u3_out);
int orc_slice_order(int64_t m, int64_t workers, uint64_t seed, int64_t sweep, int32_t *rows_out);
double orc_residual(int64_t m, const int64_t *row_ptr, const int32_t *col, const double *val, const double *b,
                    const double *x, double *r_out);
int orc_rk_run(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
               const double *b, double *x, double gamma, uint64_t seed, uint32_t stream, int sampling_uniform,
               int update_one, int64_t tau, int64_t ticket0, int64_t nsteps, int64_t curve_every,
               const double *x_ref, double *err_curve, double *res_curve, int32_t *rows_out, int slices,
               int64_t workers);
int orc_rk_apply_rows(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                      const double *b, double *x, double gamma, const int32_t *rows, const int32_t *coords,
                      int64_t count);

static uint64_t st = 88172645463325252ull;
static uint64_t next(void) {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return st;
}

static int fails = 0;
#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c);   \
            ++fails;                                                        \
        }                                                                   \
    } while (0)

int main(void) {
    int trial;
    for (trial = 0; trial < 12; ++trial) {
        const int64_t m = 1 + (int64_t)(next() % 120), n = 1 + (int64_t)(next() % 60);
        int64_t *rp = malloc((size_t)(m + 1) * sizeof *rp);
        int64_t i, k, nnz = 0;
        rp[0] = 0;
        for (i = 0; i < m; ++i) {
            int64_t len = 1 + (int64_t)(next() % (uint64_t)(n < 9 ? n : 9));
            nnz += len;
            rp[i + 1] = nnz;
        }
        int32_t *col = malloc((size_t)nnz * sizeof *col);
        double *val = malloc((size_t)nnz * sizeof *val);
        for (i = 0; i < m; ++i) {
            int64_t len = rp[i + 1] - rp[i], c0 = (int64_t)(next() % (uint64_t)n);
            for (k = 0; k < len; ++k) {
                col[rp[i] + k] = (int32_t)((c0 + k) % n);
                val[rp[i] + k] = ((double)(next() % 2001) - 1000.0) / 500.0 + 0.01;
            }
            /* sort the row's columns (insertion sort; wrap-around breaks order) */
            for (k = 1; k < len; ++k) {
                int32_t c = col[rp[i] + k];
                double v = val[rp[i] + k];
                int64_t q = k - 1;
                while (q >= 0 && col[rp[i] + q] > c) {
                    col[rp[i] + q + 1] = col[rp[i] + q];
                    val[rp[i] + q + 1] = val[rp[i] + q];
                    --q;
                }
                col[rp[i] + q + 1] = c;
                val[rp[i] + q + 1] = v;
            }
        }
        double *xs = malloc((size_t)n * sizeof *xs), *b = malloc((size_t)m * sizeof *b);
        for (i = 0; i < n; ++i) xs[i] = ((double)(next() % 1001) - 500.0) / 250.0;
        for (i = 0; i < m; ++i) {
            double acc = 0.0;
            for (k = rp[i]; k < rp[i + 1]; ++k) acc += val[k] * xs[col[k]];
            b[i] = acc;
        }
        double *w = malloc((size_t)m * sizeof *w);
        uint64_t *th = malloc((size_t)m * sizeof *th);
        int32_t *al = malloc((size_t)m * sizeof *al);
        CHECK(orc_row_weights(m, rp, val, w) < 0);
        CHECK(orc_alias_build(m, w, th, al) == 0);
        const int64_t steps = 6 * m;
        int32_t *rows = malloc((size_t)steps * sizeof *rows);
        uint32_t *u3 = malloc((size_t)steps * sizeof *u3);
        CHECK(orc_sample_rows(m, 7, 1, th, al, 5, steps, rows, u3) == 0);
        CHECK(orc_sample_rows(m, 7, 1, NULL, NULL, 0, steps, rows, NULL) == 0);
        int32_t *order = malloc((size_t)m * sizeof *order);
        CHECK(orc_slice_order(m, 1 + (int64_t)(next() % 7), 3, 2, order) == 0);
        double *x = calloc((size_t)n, sizeof *x), *r = malloc((size_t)m * sizeof *r);
        double *err = malloc(7 * sizeof *err), *res = malloc(7 * sizeof *res);
        int variant;
        for (variant = 0; variant < 5; ++variant) {
            for (i = 0; i < n; ++i) x[i] = 0.0;
            const int uniform = variant == 3, one = variant == 3, slices = variant == 4;
            const int64_t tau = variant == 1 ? 5 : 0, workers = variant == 4 ? 3 : 1;
            CHECK(orc_rk_run(m, n, rp, col, val, b, x, one ? 0.5 : 1.0, 11, 0, uniform, one, tau, slices ? 0 : 3,
                             steps, m, xs, err, res, rows, slices, workers) == 0);
            CHECK(isfinite(orc_residual(m, rp, col, val, b, x, r)));
        }
        CHECK(orc_rk_apply_rows(m, n, rp, col, val, b, x, 1.0, rows, NULL, steps) == 0);
        free(rp); free(col); free(val); free(xs); free(b); free(w); free(th); free(al);
        free(rows); free(u3); free(order); free(x); free(r); free(err); free(res);
    }
    printf("oracle sanitizer run: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
