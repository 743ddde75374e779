/* The seeded serving-stream generator run under AddressSanitizer and UBSan:
 * row lengths and contents for a spread of system sizes, including rows as
 * long as the column count.  Exit status 0 = clean run. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t sg_lengths(uint64_t seed, uint64_t req, int64_t m, int64_t n, int lo, int hi, int64_t *row_ptr);
void sg_fill(uint64_t seed, uint64_t req, int64_t m, int64_t n, const int64_t *row_ptr, int32_t *col, float *val,
             double *val64, double *x_star, double *b);

int main(void) {
    const int64_t sizes[][4] = {{1, 1, 1, 1}, {40, 8, 8, 64}, {1000, 250, 8, 64}, {3000, 40, 30, 64}, {20000, 5000, 8, 64}};
    size_t t;
    for (t = 0; t < sizeof sizes / sizeof sizes[0]; ++t) {
        const int64_t m = sizes[t][0], n = sizes[t][1];
        int64_t *rp = malloc((size_t)(m + 1) * sizeof *rp);
        const int64_t nnz = sg_lengths(4, 100 + t, m, n, (int)sizes[t][2], (int)sizes[t][3], rp);
        int32_t *col = malloc((size_t)nnz * sizeof *col);
        float *val = malloc((size_t)nnz * sizeof *val);
        double *v64 = malloc((size_t)nnz * sizeof *v64), *xs = malloc((size_t)n * sizeof *xs);
        double *b = malloc((size_t)m * sizeof *b);
        sg_fill(4, 100 + t, m, n, rp, col, val, v64, xs, b);
        int64_t i, k;
        for (i = 0; i < m; ++i)
            for (k = rp[i] + 1; k < rp[i + 1]; ++k)
                if (col[k] <= col[k - 1] || col[k] >= n) {
                    fprintf(stderr, "bad row %lld\n", (long long)i);
                    return 1;
                }
        free(rp); free(col); free(val); free(v64); free(xs); free(b);
    }
    printf("serving generator sanitizer run: ok\n");
    return 0;
}
