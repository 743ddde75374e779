/*
 * CPU oracle for the asynchronous randomized Kaczmarz method (Liu, Wright,
 * Sridhar, "An Asynchronous Parallel Randomized Kaczmarz Algorithm").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, sequential FP64
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it; the product
 * path never does.  It shares no code, header, table or constant with the
 * GPU library: the random number generator and the alias table are written
 * here a second time from their published definitions.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math), so every
 * sum below is evaluated left to right exactly as written.
 *
 * Contents
 *   orc_philox4x32_10   Philox4x32-10 counter-based generator (Salmon, Moraes,
 *                       Dror, Shaw, SC'11), used to draw the row for ticket j.
 *   orc_row_weights     w_i = ||a_i||^2 (Section 1: row i is picked with
 *                       probability ||a_i||^2 / ||A||_F^2).
 *   orc_alias_build     Walker/Vose alias table over w (Vose 1991).
 *   orc_sample_rows     ticket j -> row i(j) (and coordinate t(j)).
 *   orc_rk_run          sequential RK: eq. (2) with step length gamma,
 *                       every coordinate of the row updated (Section
 *                       "Experiments": one thread is exactly RK); optional
 *                       single-coordinate update of Algorithm 1; optional
 *                       forced read delay tau (the model k(j) >= j - tau of
 *                       eq. (3)), reading x_{j-tau} and writing x_j.
 *   orc_slice_order     one sweep's row order in the paper's experimental
 *                       scheme (row slices per worker, reshuffled each scan).
 *   orc_residual        ||b - A x||^2, sequential.
 *
 * Parity status of each function is stated on it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_ZERO_ROW 2
#define ORC_ERR_NOMEM 3

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11).  Pinned by the published known-answer
 * vectors (tests/golden/philox4x32_10_kat.txt).
 * One round: multiply words 0 and 2 by the two round multipliers, take the
 * 32-bit halves of the products, and mix with words 1, 3 and the key; the key
 * is advanced by the two Weyl increments between rounds.                    */
void orc_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    const uint32_t mul_a = 0xD2511F53u, mul_b = 0xCD9E8D57u;
    const uint32_t weyl_a = 0x9E3779B9u, weyl_b = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t pa = (uint64_t)mul_a * (uint64_t)x0;
        uint64_t pb = (uint64_t)mul_b * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)pb;
        uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)pa;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += weyl_a;
        k1 += weyl_b;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Row weights w_i = sum_k v_k^2 over the row, summed in CSR order.
 * Returns -1 if every row has w_i > 0, else the first row with w_i == 0
 * (the paper assumes A has no zero rows).                                   */
int64_t orc_row_weights(int64_t m, const int64_t *row_ptr, const double *val, double *w)
{
    int64_t i, k, bad = -1;
    for (i = 0; i < m; ++i) {
        double s = 0.0;
        for (k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s = s + val[k] * val[k];
        w[i] = s;
        if (!(s > 0.0) && bad < 0)
            bad = i;
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Vose's alias method over weights w (all > 0).
 *   W = sum w (left to right);  p_i = (w_i * m) / W
 *   work lists "small" (p < 1) and "large" (p >= 1) are filled in increasing
 *   index order and used as stacks (last in, first out).
 *   Pair s = pop(small), l = pop(large): bucket s keeps probability p_s and
 *   aliases l; then p_l <- (p_l + p_s) - 1 and l goes back on the list its
 *   new p_l belongs to.  Leftover buckets on either list keep probability 1
 *   and alias themselves.
 *   Threshold: T_k = floor(prob_k * 2^32) as an integer in [0, 2^32], with
 *   T_k = 2^32 when prob_k >= 1.
 * Pinned by: the exact reconstruction of p from (T, alias) and a chi-square
 * test of drawn rows (tests/test_oracle_sampler.py).                        */
int orc_alias_build(int64_t m, const double *w, uint64_t *thresh, int32_t *alias)
{
    double total = 0.0;
    double *p;
    int64_t *small, *large, ns = 0, nl = 0, i;
    if (m <= 0)
        return ORC_ERR_ARG;
    p = (double *)malloc((size_t)m * sizeof(double));
    small = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    large = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    if (!p || !small || !large) {
        free(p); free(small); free(large);
        return ORC_ERR_NOMEM;
    }
    for (i = 0; i < m; ++i)
        total = total + w[i];
    for (i = 0; i < m; ++i) {
        p[i] = (w[i] * (double)m) / total;
        if (p[i] < 1.0)
            small[ns++] = i;
        else
            large[nl++] = i;
    }
    while (ns > 0 && nl > 0) {
        int64_t s = small[--ns];
        int64_t l = large[--nl];
        thresh[s] = (uint64_t)(p[s] * 4294967296.0);
        alias[s] = (int32_t)l;
        p[l] = (p[l] + p[s]) - 1.0;
        if (p[l] < 1.0)
            small[ns++] = l;
        else
            large[nl++] = l;
    }
    while (nl > 0) {
        int64_t l = large[--nl];
        thresh[l] = 4294967296ull;
        alias[l] = (int32_t)l;
    }
    while (ns > 0) {
        int64_t s = small[--ns];
        thresh[s] = 4294967296ull;
        alias[s] = (int32_t)s;
    }
    free(p); free(small); free(large);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Ticket j -> row.  Counter (j mod 2^32, j div 2^32, stream, 0), key
 * (seed mod 2^32, seed div 2^32).  Bucket k = floor((u1*2^32 + u0) * m / 2^64).
 * Norm-weighted sampling (probability ||a_i||^2/||A||_F^2, Section 1): row k if
 * u2 < T_k, else alias_k.  Uniform sampling (Algorithm 1's "equal
 * probability"): row k.  u3 is returned for the single-coordinate choice of
 * Algorithm 1: position t = floor(u3 * theta_i / 2^32) inside the row.      */
typedef struct {
    uint64_t m;
    uint64_t seed;
    uint32_t stream;
    const uint64_t *thresh; /* NULL: uniform sampling */
    const int32_t *alias;
} orc_sampler;

static int64_t orc_draw(const orc_sampler *sp, int64_t ticket, uint32_t *u3)
{
    uint32_t ctr[4], key[2], u[4];
    uint64_t lo, hi, k;
    ctr[0] = (uint32_t)((uint64_t)ticket & 0xffffffffull);
    ctr[1] = (uint32_t)((uint64_t)ticket >> 32);
    ctr[2] = sp->stream;
    ctr[3] = 0u;
    key[0] = (uint32_t)(sp->seed & 0xffffffffull);
    key[1] = (uint32_t)(sp->seed >> 32);
    orc_philox4x32_10(ctr, key, u);
    lo = (uint64_t)u[0] * sp->m;
    hi = (uint64_t)u[1] * sp->m + (lo >> 32);
    k = hi >> 32;
    if (u3)
        *u3 = u[3];
    if (sp->thresh == NULL)
        return (int64_t)k;
    return ((uint64_t)u[2] < sp->thresh[k]) ? (int64_t)k : (int64_t)sp->alias[k];
}

int orc_sample_rows(int64_t m, uint64_t seed, uint32_t stream, const uint64_t *thresh,
                    const int32_t *alias, int64_t ticket0, int64_t count, int32_t *rows_out,
                    uint32_t *u3_out)
{
    orc_sampler sp;
    int64_t j;
    if (m <= 0 || m > 0x7fffffffll || count < 0)
        return ORC_ERR_ARG;
    sp.m = (uint64_t)m; sp.seed = seed; sp.stream = stream; sp.thresh = thresh; sp.alias = alias;
    for (j = 0; j < count; ++j) {
        uint32_t u3 = 0;
        rows_out[j] = (int32_t)orc_draw(&sp, ticket0 + j, &u3);
        if (u3_out)
            u3_out[j] = u3;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Row order of one sweep of the paper's experimental scheme (Section
 * "Experiments": equal row slices per thread, each slice visited in order,
 * the order reshuffled after each scan).  Worker w of R owns rows
 * [w L, min(m, (w+1) L)), L = ceil(m / R).  Its permutation for sweep s:
 * u = Philox(counter (s lo, s hi, w, 0x5C4E3D2B), key = seed); b = smallest
 * width with 2^b >= L_w, mask = 2^b - 1, h = (b + 1) / 2; position k goes
 * through  y = ((y ^ (y >> h)) * (u0 | 1) + u1) & mask,
 *          y = ((y ^ (y >> h)) * (u2 | 1) + u3) & mask
 * (32-bit wrapping arithmetic) until y < L_w.  The R workers are serialized
 * round-robin: position k of every worker before position k + 1.  Pinned by:
 * every sweep is a permutation of the rows, every slice's rows stay in their
 * slice, and the slice scheme converges to the same limit
 * (tests/test_oracle_slices.py).                                           */
static uint32_t orc_slice_perm(uint32_t k, uint32_t len, const uint32_t *u)
{
    uint32_t width = 0, mask, half, y = k;
    if (len <= 1)
        return 0;
    while (width < 32 && ((uint64_t)1 << width) < (uint64_t)len)
        ++width;
    mask = width >= 32 ? 0xffffffffu : (uint32_t)(((uint64_t)1 << width) - 1u);
    half = (width + 1) / 2;
    do {
        y = ((y ^ (y >> half)) * (u[0] | 1u) + u[1]) & mask;
        y = ((y ^ (y >> half)) * (u[2] | 1u) + u[3]) & mask;
    } while (y >= len);
    return y;
}

int orc_slice_order(int64_t m, int64_t workers, uint64_t seed, int64_t sweep, int32_t *rows_out)
{
    int64_t L, w, k, q = 0, kmax;
    uint32_t key[2];
    uint32_t *u;
    if (m <= 0 || workers <= 0)
        return ORC_ERR_ARG;
    L = (m + workers - 1) / workers;
    key[0] = (uint32_t)(seed & 0xffffffffull);
    key[1] = (uint32_t)(seed >> 32);
    u = (uint32_t *)malloc((size_t)workers * 4 * sizeof(uint32_t));
    if (!u)
        return ORC_ERR_NOMEM;
    for (w = 0; w < workers; ++w) {
        uint32_t ctr[4];
        ctr[0] = (uint32_t)((uint64_t)sweep & 0xffffffffull);
        ctr[1] = (uint32_t)((uint64_t)sweep >> 32);
        ctr[2] = (uint32_t)w;
        ctr[3] = 0x5C4E3D2Bu;
        orc_philox4x32_10(ctr, key, u + 4 * w);
    }
    kmax = L;
    for (k = 0; k < kmax; ++k) {
        for (w = 0; w < workers; ++w) {
            int64_t start = w * L, len;
            if (start >= m)
                continue;
            len = (m - start < L) ? m - start : L;
            if (k >= len)
                continue;
            rows_out[q++] = (int32_t)(start + orc_slice_perm((uint32_t)k, (uint32_t)len, u + 4 * w));
        }
    }
    free(u);
    return q == m ? ORC_OK : ORC_ERR_ARG;
}

/* ------------------------------------------------------------------------ */
/* ||b - A x||^2 with r_i = b_i - sum_k v_k x_{c_k} (CSR order), summed over i
 * in order.  r_out may be NULL.  Pinned against scipy's sparse product.     */
double orc_residual(int64_t m, const int64_t *row_ptr, const int32_t *col, const double *val,
                    const double *b, const double *x, double *r_out)
{
    double acc = 0.0;
    int64_t i, k;
    for (i = 0; i < m; ++i) {
        double p = 0.0, r;
        for (k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            p = p + val[k] * x[col[k]];
        r = b[i] - p;
        if (r_out)
            r_out[i] = r;
        acc = acc + r * r;
    }
    return acc;
}

static double orc_rel_err(int64_t n, const double *x, const double *xr)
{
    double num = 0.0, den = 0.0;
    int64_t c;
    for (c = 0; c < n; ++c) {
        double d = x[c] - xr[c];
        num = num + d * d;
        den = den + xr[c] * xr[c];
    }
    return den > 0.0 ? sqrt(num / den) : sqrt(num);
}

/* ------------------------------------------------------------------------ */
/* Sequential RK run.
 *
 * For tickets j = ticket0 ... ticket0 + nsteps - 1:
 *   i = row drawn for j (norm-weighted or uniform, see orc_draw)
 *   p = sum_k v_k * xr_{c_k}     xr = x_j when tau == 0, else x_{max(ticket0, j - tau)}
 *   r = p - b_i
 *   update_all (eq. (2) with step length gamma, all coordinates):
 *       s = (gamma * r) / w_i ;  x_{c_k} <- x_{c_k} - s * v_k  for every k, in CSR order
 *   update_one (Algorithm 1, coordinate t = floor(u3 * theta_i / 2^32)):
 *       s = ((gamma * theta_i) * r) / w_i ;  x_{c_t} <- x_{c_t} - s * v_t
 * (The paper normalizes rows, w_i = 1; dividing by w_i keeps the projection
 * exact for rows that are not exactly unit length.)
 *
 * Curves: if curve_every > 0, after step 0 and after every curve_every steps,
 * err_curve[q] = ||x - x_ref|| / ||x_ref|| (when x_ref != NULL) and
 * res_curve[q] = ||A x - b|| / ||b||.  rows_out (nullable) receives every row.
 *
 * Pinned by: closed forms (one-row system, identity rows), the per-step
 * projection and Pythagorean identities, the exact one-step expectation, the
 * expected-rate bound of Section 1 and convergence to the least-squares
 * solution (tests/test_oracle_rk.py).  The delayed read (tau > 0) reduces to
 * the tau = 0 run bit for bit and is otherwise pinned only by its own
 * convergence checks.
 * ------------------------------------------------------------------------ */
int orc_rk_run(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
               const double *val, const double *b, double *x, double gamma,
               uint64_t seed, uint32_t stream, int sampling_uniform, int update_one,
               int64_t tau, int64_t ticket0, int64_t nsteps, int64_t curve_every,
               const double *x_ref, double *err_curve, double *res_curve, int32_t *rows_out,
               int slices, int64_t workers)
{
    double *w = NULL, *corr = NULL, *pend_s = NULL;
    int32_t *sweep_rows = NULL;
    uint64_t *thresh = NULL;
    int32_t *alias = NULL, *mark = NULL;
    int64_t *pend_row = NULL, *pend_t = NULL;
    double bnorm = 0.0;
    orc_sampler sp;
    int64_t j, q = 0, npend = 0, head = 0;
    int rc = ORC_OK;

    if (m <= 0 || n <= 0 || m > 0x7fffffffll || n > 0x7fffffffll || nsteps < 0 || tau < 0 || !(gamma > 0.0))
        return ORC_ERR_ARG;
    if (slices && (update_one || workers <= 0 || ticket0 % m != 0))
        return ORC_ERR_ARG;
    w = (double *)malloc((size_t)m * sizeof(double));
    if (!w)
        return ORC_ERR_NOMEM;
    if (orc_row_weights(m, row_ptr, val, w) >= 0) {
        free(w);
        return ORC_ERR_ZERO_ROW;
    }
    sp.m = (uint64_t)m; sp.seed = seed; sp.stream = stream; sp.thresh = NULL; sp.alias = NULL;
    if (!sampling_uniform) {
        thresh = (uint64_t *)malloc((size_t)m * sizeof(uint64_t));
        alias = (int32_t *)malloc((size_t)m * sizeof(int32_t));
        if (!thresh || !alias) { rc = ORC_ERR_NOMEM; goto done; }
        rc = orc_alias_build(m, w, thresh, alias);
        if (rc != ORC_OK) goto done;
        sp.thresh = thresh; sp.alias = alias;
    }
    if (tau > 0) {
        int64_t maxnnz = 0, i;
        for (i = 0; i < m; ++i)
            if (row_ptr[i + 1] - row_ptr[i] > maxnnz) maxnnz = row_ptr[i + 1] - row_ptr[i];
        corr = (double *)calloc((size_t)(maxnnz + 1), sizeof(double));
        mark = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        pend_s = (double *)malloc((size_t)tau * sizeof(double));
        pend_row = (int64_t *)malloc((size_t)tau * sizeof(int64_t));
        pend_t = (int64_t *)malloc((size_t)tau * sizeof(int64_t));
        if (!corr || !mark || !pend_s || !pend_row || !pend_t) { rc = ORC_ERR_NOMEM; goto done; }
        for (i = 0; i < n; ++i) mark[i] = -1;
    }
    if (curve_every > 0) {
        int64_t i;
        for (i = 0; i < m; ++i) bnorm = bnorm + b[i] * b[i];
        bnorm = sqrt(bnorm);
        if (x_ref && err_curve) err_curve[0] = orc_rel_err(n, x, x_ref);
        if (res_curve) {
            double r2 = orc_residual(m, row_ptr, col, val, b, x, NULL);
            res_curve[0] = bnorm > 0.0 ? sqrt(r2) / bnorm : sqrt(r2);
        }
    }

    if (slices) {
        sweep_rows = (int32_t *)malloc((size_t)m * sizeof(int32_t));
        if (!sweep_rows) { rc = ORC_ERR_NOMEM; goto done; }
    }
    for (j = 0; j < nsteps; ++j) {
        uint32_t u3 = 0;
        int64_t i;
        if (slices) {
            int64_t t = ticket0 + j;
            if (j == 0 || t % m == 0) {
                rc = orc_slice_order(m, workers, seed, t / m, sweep_rows);
                if (rc != ORC_OK) goto done;
            }
            i = sweep_rows[t % m];
        } else {
            i = orc_draw(&sp, ticket0 + j, &u3);
        }
        int64_t beg = row_ptr[i], end = row_ptr[i + 1], k;
        double p = 0.0, r, s;
        if (rows_out) rows_out[j] = (int32_t)i;
        if (tau > 0 && npend > 0) {
            /* x_{j - tau} on supp(a_i): undo the pending (not yet visible)
             * updates, oldest first. */
            int64_t e;
            for (k = beg; k < end; ++k) { mark[col[k]] = (int32_t)(k - beg); corr[k - beg] = 0.0; }
            for (e = 0; e < npend; ++e) {
                int64_t slot = (head + e) % tau;
                int64_t pr = pend_row[slot], kk;
                if (pend_t[slot] >= 0) {
                    kk = row_ptr[pr] + pend_t[slot];
                    if (mark[col[kk]] >= 0) corr[mark[col[kk]]] = corr[mark[col[kk]]] + pend_s[slot] * val[kk];
                } else {
                    for (kk = row_ptr[pr]; kk < row_ptr[pr + 1]; ++kk)
                        if (mark[col[kk]] >= 0)
                            corr[mark[col[kk]]] = corr[mark[col[kk]]] + pend_s[slot] * val[kk];
                }
            }
            for (k = beg; k < end; ++k) {
                p = p + val[k] * (x[col[k]] + corr[k - beg]);
                mark[col[k]] = -1;
            }
        } else {
            for (k = beg; k < end; ++k)
                p = p + val[k] * x[col[k]];
        }
        r = p - b[i];
        if (!update_one) {
            s = (gamma * r) / w[i];
            for (k = beg; k < end; ++k)
                x[col[k]] = x[col[k]] - s * val[k];
        } else {
            int64_t theta = end - beg;
            int64_t t = (int64_t)(((uint64_t)u3 * (uint64_t)theta) >> 32);
            s = ((gamma * (double)theta) * r) / w[i];
            x[col[beg + t]] = x[col[beg + t]] - s * val[beg + t];
        }
        if (tau > 0) {
            /* remember this update; it stays invisible to the next tau reads */
            int64_t slot;
            if (npend == tau) { head = (head + 1) % tau; npend--; }
            slot = (head + npend) % tau;
            pend_row[slot] = i;
            pend_s[slot] = s;
            pend_t[slot] = update_one ? (int64_t)(((uint64_t)u3 * (uint64_t)(end - beg)) >> 32) : -1;
            npend++;
        }
        if (curve_every > 0 && (j + 1) % curve_every == 0) {
            ++q;
            if (x_ref && err_curve) err_curve[q] = orc_rel_err(n, x, x_ref);
            if (res_curve) {
                double r2 = orc_residual(m, row_ptr, col, val, b, x, NULL);
                res_curve[q] = bnorm > 0.0 ? sqrt(r2) / bnorm : sqrt(r2);
            }
        }
    }
done:
    free(sweep_rows);
    free(w); free(thresh); free(alias); free(corr); free(mark);
    free(pend_s); free(pend_row); free(pend_t);
    return rc;
}

/* Rows (and, for Algorithm 1's step, coordinates) applied in the given order,
 * with no sampling: the same update as orc_rk_run with tau = 0, for tests
 * that enumerate every row or every (row, coordinate) pair.  coords may be
 * NULL (every coordinate of each row); coords[j] >= 0 selects position t of
 * row rows[j] and applies the single-coordinate step with the theta factor. */
int orc_rk_apply_rows(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
                      const double *val, const double *b, double *x, double gamma,
                      const int32_t *rows, const int32_t *coords, int64_t count)
{
    int64_t j;
    (void)n;
    for (j = 0; j < count; ++j) {
        int64_t i = rows[j], k, beg, end;
        double p = 0.0, w = 0.0, r, s;
        if (i < 0 || i >= m) return ORC_ERR_ARG;
        beg = row_ptr[i]; end = row_ptr[i + 1];
        for (k = beg; k < end; ++k) w = w + val[k] * val[k];
        if (!(w > 0.0)) return ORC_ERR_ZERO_ROW;
        for (k = beg; k < end; ++k) p = p + val[k] * x[col[k]];
        r = p - b[i];
        if (coords == NULL || coords[j] < 0) {
            s = (gamma * r) / w;
            for (k = beg; k < end; ++k) x[col[k]] = x[col[k]] - s * val[k];
        } else {
            int64_t theta = end - beg, t = coords[j];
            if (t >= theta) return ORC_ERR_ARG;
            s = ((gamma * (double)theta) * r) / w;
            x[col[beg + t]] = x[col[beg + t]] - s * val[beg + t];
        }
    }
    return ORC_OK;
}
