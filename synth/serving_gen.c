/*
 * Fast seeded generator for the serving stream's systems (input data only).
 *
 * One request (seed, request_id, m, n): row lengths uniform in [lo, hi]
 * (capped at n), distinct uniform columns per row (rejection against a
 * bitmap of the row's earlier draws), sorted ascending; N(0,1) values
 * (Marsaglia's polar method), each row
 * scaled to unit norm in FP64 and rounded to FP32; x* ~ N(0,1); b = A x* in
 * FP64 from the FP32 values.  Random numbers: xoshiro256** seeded by
 * splitmix64 from (seed, request_id, substream): substream 0 for lengths,
 * 1 for everything else.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s[4]; } xo_state;

static uint64_t splitmix64(uint64_t *x)
{
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void xo_seed(xo_state *st, uint64_t seed, uint64_t req, uint64_t sub)
{
    uint64_t x = seed * 0x100000001B3ull ^ (req + 0x632BE59BD9B4E019ull) ^ (sub << 56);
    int i;
    for (i = 0; i < 4; ++i) st->s[i] = splitmix64(&x);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t xo_next(xo_state *st)
{
    uint64_t *s = st->s;
    uint64_t r = rotl(s[1] * 5, 7) * 9, t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return r;
}

/* uniform integer in [0, bound) (Lemire's multiply-shift, bias < 2^-32 for bound < 2^32) */
static inline uint64_t xo_below(xo_state *st, uint64_t bound)
{
    return (uint64_t)(((unsigned __int128)xo_next(st) * bound) >> 64);
}

static inline double xo_unit(xo_state *st) { return ((xo_next(st) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

/* N(0,1) by Marsaglia's polar method (pairs; the second value is kept) */
static double xo_normal(xo_state *st, double *spare, int *have)
{
    double u, v, q, f;
    if (*have) { *have = 0; return *spare; }
    do {
        u = 2.0 * xo_unit(st) - 1.0;
        v = 2.0 * xo_unit(st) - 1.0;
        q = u * u + v * v;
    } while (q >= 1.0 || q == 0.0);
    f = sqrt(-2.0 * log(q) / q);
    *spare = v * f;
    *have = 1;
    return u * f;
}

/* Row lengths (row_ptr[0..m]); returns nnz. */
int64_t sg_lengths(uint64_t seed, uint64_t req, int64_t m, int64_t n, int lo, int hi, int64_t *row_ptr)
{
    xo_state st;
    int64_t i;
    if (hi > n) hi = (int)n;
    if (lo > hi) lo = hi;
    xo_seed(&st, seed, req, 0);
    row_ptr[0] = 0;
    for (i = 0; i < m; ++i)
        row_ptr[i + 1] = row_ptr[i] + lo + (int64_t)xo_below(&st, (uint64_t)(hi - lo + 1));
    return row_ptr[m];
}

/* Columns, values, x* and b for the lengths in row_ptr. */
void sg_fill(uint64_t seed, uint64_t req, int64_t m, int64_t n, const int64_t *row_ptr,
             int32_t *col, float *val, double *val64, double *x_star, double *b)
{
    xo_state st;
    double spare = 0.0;
    int have = 0;
    int64_t i, c;
    uint64_t *seen = (uint64_t *)calloc((size_t)((n + 63) / 64), sizeof(uint64_t));
    xo_seed(&st, seed, req, 1);
    for (i = 0; i < m; ++i) {
        int64_t beg = row_ptr[i], k = row_ptr[i + 1] - beg, a, q;
        double nrm = 0.0;
        for (a = 0; a < k; ++a) {
            int32_t v;
            do {
                v = (int32_t)xo_below(&st, (uint64_t)n);
            } while (seen[v >> 6] & (1ull << (v & 63)));
            seen[v >> 6] |= 1ull << (v & 63);
            col[beg + a] = v;
        }
        for (a = 0; a < k; ++a) seen[col[beg + a] >> 6] &= ~(1ull << (col[beg + a] & 63));
        /* insertion sort of the row's columns */
        for (a = 1; a < k; ++a) {
            int32_t v = col[beg + a];
            q = a - 1;
            while (q >= 0 && col[beg + q] > v) { col[beg + q + 1] = col[beg + q]; --q; }
            col[beg + q + 1] = v;
        }
        for (a = 0; a < k; ++a) {
            double g = xo_normal(&st, &spare, &have);
            val64[beg + a] = g;
            nrm += g * g;
        }
        nrm = sqrt(nrm);
        for (a = 0; a < k; ++a) {
            val[beg + a] = (float)(val64[beg + a] / nrm);
            val64[beg + a] = (double)val[beg + a];
        }
    }
    free(seen);
    for (c = 0; c < n; ++c) x_star[c] = xo_normal(&st, &spare, &have);
    for (i = 0; i < m; ++i) {
        double s = 0.0;
        int64_t k;
        for (k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += val64[k] * x_star[col[k]];
        b[i] = s;
    }
}
