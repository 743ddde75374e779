// Host-side system setup: CSR validation, row weights, alias table and row
// record packing.  Plain C++ compiled with -ffp-contract=off so the FP64
// weights and the alias table follow the sampling rule of the C ABI exactly
// (every sum left to right, no fused multiply-add).
#include "setup.h"

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace asyrk {

static inline double promote(const void *vals, int vk, int64_t k) {
    switch (vk) {
        case ASYRK_F64: return static_cast<const double *>(vals)[k];
        case ASYRK_F32: return (double)static_cast<const float *>(vals)[k];
        default: {
            const uint32_t u = (uint32_t) static_cast<const uint16_t *>(vals)[k] << 16;
            float f;
            std::memcpy(&f, &u, 4);
            return (double)f;
        }
    }
}

template <class F>
static void parallel_rows(int64_t m, F fn) {
    unsigned nt = std::thread::hardware_concurrency();
    nt = std::max(1u, std::min(nt, 16u));
    if (m < 65536) nt = 1;
    std::vector<std::thread> th;
    const int64_t chunk = (m + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t lo = t * chunk, hi = std::min<int64_t>(m, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([=]() { fn(lo, hi); });
    }
    for (auto &x : th) x.join();
}

// Validation of A and b; fills the row weights w_i = ||a_i||^2 (FP64 from the
// stored values, summed in CSR order) and the column-count statistics.
asyrk_status validate_system(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const void *vals, int vk, const double *b, SetupResult &out) {
    if (m < 1 || n < 1 || m > INT32_MAX || n > INT32_MAX) return ASYRK_ERR_INVALID_ARG;
    if (vk != ASYRK_F64 && vk != ASYRK_F32 && vk != ASYRK_BF16) return ASYRK_ERR_INVALID_ARG;
    if (!row_ptr || !b) return ASYRK_ERR_INVALID_ARG;
    if (row_ptr[0] != 0) return ASYRK_ERR_INVALID_ARG;
    for (int64_t i = 0; i < m; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return ASYRK_ERR_INVALID_ARG;
    const int64_t nnz = row_ptr[m];
    if (nnz >= (int64_t)INT32_MAX) return ASYRK_ERR_INVALID_ARG;
    if (nnz > 0 && (!col || !vals)) return ASYRK_ERR_INVALID_ARG;
    for (int64_t i = 0; i < m; ++i)
        if (!std::isfinite(b[i])) return ASYRK_ERR_INVALID_ARG;

    out.w.assign(m, 0.0);
    std::vector<int> bad_t(16, 0);
    std::vector<int64_t> mu_t(16, 0);
    int tix = 0;
    std::vector<std::pair<int64_t, int64_t>> ranges;
    {
        unsigned nt = std::max(1u, std::min(std::thread::hardware_concurrency(), 16u));
        if (m < 65536) nt = 1;
        const int64_t chunk = (m + nt - 1) / nt;
        for (unsigned t = 0; t < nt; ++t) {
            const int64_t lo = t * chunk, hi = std::min<int64_t>(m, lo + chunk);
            if (lo < hi) ranges.emplace_back(lo, hi);
        }
    }
    std::vector<std::thread> th;
    for (auto &rg : ranges) {
        const int me = tix++;
        th.emplace_back([&, me, rg]() {
            int64_t mu = 0;
            for (int64_t i = rg.first; i < rg.second; ++i) {
                const int64_t beg = row_ptr[i], end = row_ptr[i + 1];
                mu = std::max(mu, end - beg);
                double s = 0.0;
                int32_t prev = -1;
                for (int64_t k = beg; k < end; ++k) {
                    const int32_t c = col[k];
                    if (c <= prev || c >= n) { bad_t[me] = 1; return; }
                    prev = c;
                    const double v = promote(vals, vk, k);
                    if (!std::isfinite(v)) { bad_t[me] = 1; return; }
                    s = s + v * v;
                }
                out.w[i] = s;
            }
            mu_t[me] = mu;
        });
    }
    for (auto &x : th) x.join();
    for (int t = 0; t < tix; ++t)
        if (bad_t[t]) return ASYRK_ERR_INVALID_ARG;
    for (int64_t i = 0; i < m; ++i)
        if (!(out.w[i] > 0.0)) return ASYRK_ERR_ZERO_ROW;

    out.mu = 0;
    for (int t = 0; t < tix; ++t) out.mu = std::max(out.mu, mu_t[t]);
    std::vector<int32_t> cnt(n, 0);
    std::vector<double> cn2(n, 0.0);
    for (int64_t k = 0; k < nnz; ++k) {
        const double v = promote(vals, vk, k);
        cnt[col[k]]++;
        cn2[col[k]] += v * v;
    }
    out.nu = *std::max_element(cnt.begin(), cnt.end());
    out.max_col_norm2 = *std::max_element(cn2.begin(), cn2.end());
    out.fixed_nnz = row_ptr[1] - row_ptr[0];
    for (int64_t i = 1; i < m && out.fixed_nnz > 0; ++i)
        if (row_ptr[i + 1] - row_ptr[i] != out.fixed_nnz) out.fixed_nnz = 0;
    double fro2 = 0.0;
    for (int64_t i = 0; i < m; ++i) fro2 = fro2 + out.w[i];
    out.fro2 = fro2;
    out.nnz = nnz;
    return ASYRK_OK;
}

// Vose's alias method for P(i) = w_i / sum(w): p_i = (w_i m) / W with W
// summed left to right; the small (p < 1) and large (p >= 1) work lists are
// filled in increasing index order and used last-in first-out; pairing
// (s, l) gives bucket s threshold floor(p_s 2^32) and alias l, then
// p_l <- (p_l + p_s) - 1.  Buckets left on either list keep their own row
// (threshold stored as 2^32 - 1 with alias = itself, which selects the
// bucket's row for every u2).
void build_alias(const std::vector<double> &w, std::vector<uint32_t> &thresh,
                 std::vector<int32_t> &alias) {
    const int64_t m = (int64_t)w.size();
    double total = 0.0;
    for (int64_t i = 0; i < m; ++i) total = total + w[i];
    std::vector<double> p(m);
    std::vector<int64_t> small, large;
    small.reserve(m);
    large.reserve(m);
    for (int64_t i = 0; i < m; ++i) {
        p[i] = (w[i] * (double)m) / total;
        if (p[i] < 1.0)
            small.push_back(i);
        else
            large.push_back(i);
    }
    thresh.assign(m, 0xffffffffu);
    alias.resize(m);
    for (int64_t i = 0; i < m; ++i) alias[i] = (int32_t)i;
    while (!small.empty() && !large.empty()) {
        const int64_t s = small.back();
        small.pop_back();
        const int64_t l = large.back();
        large.pop_back();
        thresh[s] = (uint32_t)(uint64_t)(p[s] * 4294967296.0);
        alias[s] = (int32_t)l;
        p[l] = (p[l] + p[s]) - 1.0;
        if (p[l] < 1.0)
            small.push_back(l);
        else
            large.push_back(l);
    }
    // leftovers keep thresh = 2^32 - 1 and alias = self
}

// Store a FP64 value in the dtype (BF16: nearest, ties to even, of the FP32 value).
static void store_as(double v, int vk, uint8_t *dst) {
    if (vk == ASYRK_F64) {
        std::memcpy(dst, &v, 8);
    } else {
        const float f = (float)v;
        if (vk == ASYRK_F32) {
            std::memcpy(dst, &f, 4);
        } else {
            uint32_t u;
            std::memcpy(&u, &f, 4);
            const uint32_t bias = ((u >> 16) & 1u) + 0x7FFFu;
            const uint16_t h = (uint16_t)((u + bias) >> 16);
            std::memcpy(dst, &h, 2);
        }
    }
}

// Rows 0..n-1: row j holds phi * A[i, j] at columns n + i (i increasing) and
// right-hand side phi * sum_i A[i, j] b_i (i increasing); rows n..n+m-1: row
// n + i holds a_i at its own columns, then -zeta at column n + i, right-hand
// side 0.
asyrk_status build_augmented(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const void *vals, int vk, const double *b, double zeta, double phi, AugCSR &out) {
    if (!(zeta > 0.0) || !(phi > 0.0) || !std::isfinite(zeta) || !std::isfinite(phi)) return ASYRK_ERR_INVALID_ARG;
    if (m < 1 || n < 1 || m + n > INT32_MAX) return ASYRK_ERR_INVALID_ARG;
    const int64_t nnz = row_ptr[m];
    if (2 * nnz + m >= (int64_t)INT32_MAX) return ASYRK_ERR_INVALID_ARG;
    const int vb = vk == ASYRK_F64 ? 8 : (vk == ASYRK_F32 ? 4 : 2);
    const int64_t N = n + m;
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) cnt[col[k] + 1]++;
    for (int64_t j = 0; j < n; ++j)
        if (cnt[j + 1] == 0) return ASYRK_ERR_ZERO_ROW;  // an empty column of A
    for (int64_t j = 0; j < n; ++j) cnt[j + 1] += cnt[j];
    try {
        out.row_ptr.assign(N + 1, 0);
        out.col.resize(2 * nnz + m);
        out.vals.resize((2 * nnz + m) * vb);
        out.b.assign(N, 0.0);
    } catch (...) {
        return ASYRK_ERR_OOM;
    }
    for (int64_t j = 0; j < n; ++j) out.row_ptr[j + 1] = cnt[j + 1];
    for (int64_t i = 0; i < m; ++i) out.row_ptr[n + i + 1] = nnz + row_ptr[i + 1] + i + 1;
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    std::vector<double> atb(n, 0.0);
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const int32_t j = col[k];
            const double a = promote(vals, vk, k);
            const int64_t pos = fill[j]++;
            out.col[pos] = (int32_t)(n + i);
            store_as(phi * a, vk, &out.vals[pos * vb]);
            atb[j] = atb[j] + a * b[i];
        }
        const int64_t base = nnz + row_ptr[i] + i;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            out.col[base + (k - row_ptr[i])] = col[k];
            std::memcpy(&out.vals[(base + (k - row_ptr[i])) * vb], static_cast<const uint8_t *>(vals) + k * vb, vb);
        }
        const int64_t last = nnz + row_ptr[i + 1] + i;
        out.col[last] = (int32_t)(n + i);
        store_as(-zeta, vk, &out.vals[last * vb]);
    }
    for (int64_t j = 0; j < n; ++j) out.b[j] = phi * atb[j];
    return ASYRK_OK;
}

// Record stride for equal-length rows: pad to 64 bytes when that touches
// fewer 64-byte sectors per record than 16-byte packing does on average.
static int64_t choose_stride(int64_t raw) {
    double avg16 = 0.0;
    for (int r = 0; r < 4; ++r) {
        const int64_t o = (r * raw) % 64;
        avg16 += (double)((o + raw + 63) / 64);
    }
    avg16 /= 4.0;
    const int64_t pad64 = (raw + 63) / 64 * 64;
    const double sec64 = (double)(pad64 / 64);
    return sec64 <= avg16 - 1e-9 ? pad64 : raw;
}

asyrk_status pack_records(int64_t m, const int64_t *row_ptr, const int32_t *col, const void *vals,
                          int vk, const double *b, SetupResult &res) {
    const Geom g = geom_of(vk);
    std::vector<uint32_t> thresh;
    std::vector<int32_t> alias;
    build_alias(res.w, thresh, alias);

    auto raw_bytes = [&](int64_t nnz) { return (int64_t)g.HB + (nnz + g.U - 1) / g.U * g.UB; };
    std::vector<int64_t> off;
    int64_t total;
    if (res.fixed_nnz > 0) {
        res.stride = choose_stride(raw_bytes(res.fixed_nnz));
        total = res.stride * m;
    } else {
        res.stride = 0;
        off.resize(m + 1);
        off[0] = 0;
        for (int64_t i = 0; i < m; ++i) off[i + 1] = off[i] + raw_bytes(row_ptr[i + 1] - row_ptr[i]);
        total = off[m];
        if (total / 16 >= (int64_t)UINT32_MAX) return ASYRK_ERR_INVALID_ARG;
        res.loc.resize(m);
        for (int64_t i = 0; i < m; ++i)
            res.loc[i] = RowLoc{(uint32_t)(off[i] / 16), (uint32_t)(row_ptr[i + 1] - row_ptr[i])};
    }
    try {
        res.rec.assign((size_t)total, 0);
    } catch (...) {
        return ASYRK_ERR_OOM;
    }
    uint8_t *base = res.rec.data();
    const std::vector<double> &w = res.w;
    parallel_rows(m, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            uint8_t *r = base + (res.fixed_nnz > 0 ? i * res.stride : off[i]);
            const double inv_w = 1.0 / w[i];
            if (vk == ASYRK_F64) {
                HdrF64 h{b[i], inv_w, thresh[i], alias[i], 0};
                std::memcpy(r, &h, sizeof h);
            } else {
                HdrF32 h{(float)b[i], (float)inv_w, thresh[i], alias[i]};
                std::memcpy(r, &h, sizeof h);
            }
            const int64_t beg = row_ptr[i], nnz = row_ptr[i + 1] - beg;
            for (int64_t k = 0; k < nnz; ++k) {
                uint8_t *u = r + g.HB + (k / g.U) * g.UB;
                const int e = (int)(k % g.U);
                std::memcpy(u + 4 * e, &col[beg + k], 4);
                std::memcpy(u + g.COLB + g.VB * e, static_cast<const uint8_t *>(vals) + (beg + k) * g.VB,
                            g.VB);
            }
        }
    });
    return ASYRK_OK;
}

}  // namespace asyrk
