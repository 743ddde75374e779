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
#include <memory>
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

// Host threads for a pass over m rows: one per 4096 rows, at most 16 and at
// most the hardware's.
static unsigned threads_for(int64_t m) {
    const unsigned hw = std::max(1u, std::min(std::thread::hardware_concurrency(), 16u));
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(hw, m / 4096));
}

// fn(lo, hi) over `parts` contiguous row ranges, the first on the calling thread.
template <class F>
static void parallel_rows(int64_t m, unsigned parts, F fn) {
    if (parts <= 1) {
        fn((int64_t)0, m);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (m + parts - 1) / parts;
    for (unsigned t = 1; t < parts; ++t) {
        const int64_t lo = t * chunk, hi = std::min<int64_t>(m, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([=]() { fn(lo, hi); });
    }
    fn((int64_t)0, std::min<int64_t>(m, chunk));
    for (auto &x : th) x.join();
}

template <int VK>
static inline double promote_t(const void *vals, int64_t k) {
    if constexpr (VK == ASYRK_F64) {
        return static_cast<const double *>(vals)[k];
    } else if constexpr (VK == ASYRK_F32) {
        return (double)static_cast<const float *>(vals)[k];
    } else {
        const uint32_t u = (uint32_t) static_cast<const uint16_t *>(vals)[k] << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return (double)f;
    }
}

// Rows lo..hi-1: sorted in-range columns, finite values, w_i (FP64, CSR
// order).  With cs the column statistics are accumulated in the same pass
// (entries in increasing k, as the separate pass would).  Returns false on an
// invalid entry.
// Per-column entry count and sum of squares, side by side (one cache line per update).
struct ColStat {
    double sq;
    int64_t cnt;
};

template <int VK>
static bool scan_rows(int64_t lo, int64_t hi, int64_t n, const int64_t *row_ptr, const int32_t *col,
                      const void *vals, double *w, int64_t &mu_out, ColStat *cs) {
    int64_t mu = 0;
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t beg = row_ptr[i], end = row_ptr[i + 1];
        mu = std::max(mu, end - beg);
        double s = 0.0;
        int32_t prev = -1;
        for (int64_t k = beg; k < end; ++k) {
            const int32_t c = col[k];
            if (c <= prev || c >= n) return false;
            prev = c;
            const double v = promote_t<VK>(vals, k);
            if (!std::isfinite(v)) return false;
            const double v2 = v * v;
            s = s + v2;
            if (cs) {
                cs[c].cnt++;
                cs[c].sq += v2;
            }
        }
        w[i] = s;
    }
    mu_out = mu;
    return true;
}

template <int VK>
static asyrk_status validate_t(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col, const void *vals,
                               SetupResult &out) {
    const int64_t nnz = row_ptr[m];
    out.w.resize(m);
    std::vector<ColStat> cs(n, ColStat{0.0, 0});
    const unsigned nt = threads_for(m);
    int64_t mu = 0;
    if (nt == 1) {
        if (!scan_rows<VK>(0, m, n, row_ptr, col, vals, out.w.data(), mu, cs.data()))
            return ASYRK_ERR_INVALID_ARG;
    } else {
        // nt - 1 threads scan row ranges while the calling thread accumulates
        // the column statistics over every entry in order (the same sums as
        // the single-threaded pass), checking each index against n itself
        // since the row scan runs at the same time.
        const unsigned parts = nt - 1;
        std::vector<int> bad(parts, 0);
        std::vector<int64_t> mu_t(parts, 0);
        std::vector<std::thread> th;
        const int64_t chunk = (m + parts - 1) / parts;
        for (unsigned t = 0; t < parts; ++t) {
            const int64_t lo = t * chunk, hi = std::min<int64_t>(m, lo + chunk);
            if (lo >= hi) break;
            th.emplace_back([&, t, lo, hi]() {
                bad[t] = !scan_rows<VK>(lo, hi, n, row_ptr, col, vals, out.w.data(), mu_t[t], nullptr);
            });
        }
        bool in_range = true;
        for (int64_t k = 0; k < nnz; ++k) {
            const int32_t c = col[k];
            if (c < 0 || c >= n) {
                in_range = false;
                break;
            }
            const double v = promote_t<VK>(vals, k);
            cs[c].cnt++;
            cs[c].sq += v * v;
        }
        for (auto &x : th) x.join();
        for (unsigned t = 0; t < parts; ++t) {
            if (bad[t]) return ASYRK_ERR_INVALID_ARG;
            mu = std::max(mu, mu_t[t]);
        }
        if (!in_range) return ASYRK_ERR_INVALID_ARG;
    }
    for (int64_t i = 0; i < m; ++i)
        if (!(out.w[i] > 0.0)) return ASYRK_ERR_ZERO_ROW;
    out.mu = mu;
    out.nu = 0;
    out.max_col_norm2 = cs[0].sq;
    for (const ColStat &c : cs) {
        out.nu = std::max(out.nu, c.cnt);
        out.max_col_norm2 = std::max(out.max_col_norm2, c.sq);
    }
    out.fixed_nnz = row_ptr[1] - row_ptr[0];
    for (int64_t i = 1; i < m && out.fixed_nnz > 0; ++i)
        if (row_ptr[i + 1] - row_ptr[i] != out.fixed_nnz) out.fixed_nnz = 0;
    double fro2 = 0.0;
    for (int64_t i = 0; i < m; ++i) fro2 = fro2 + out.w[i];
    out.fro2 = fro2;
    out.nnz = nnz;
    return ASYRK_OK;
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
    switch (vk) {
        case ASYRK_F64: return validate_t<ASYRK_F64>(m, n, row_ptr, col, vals, out);
        case ASYRK_F32: return validate_t<ASYRK_F32>(m, n, row_ptr, col, vals, out);
        default: return validate_t<ASYRK_BF16>(m, n, row_ptr, col, vals, out);
    }
}

// Vose's alias method for P(i) = w_i / sum(w): p_i = (w_i m) / W with W
// summed left to right; the small (p < 1) and large (p >= 1) work lists are
// filled in increasing index order and used last-in first-out; pairing
// (s, l) gives bucket s threshold floor(p_s 2^32) and alias l, then
// p_l <- (p_l + p_s) - 1.  Buckets left on either list keep their own row
// (threshold stored as 2^32 - 1 with alias = itself, which selects the
// bucket's row for every u2).
void build_alias(const double *w, int64_t m, double total, uint32_t *thresh, int32_t *alias) {
    std::unique_ptr<double[]> p(new double[m]);
    // Both work lists share one array: the small list grows up from the
    // front, the large list down from the back (each index is on at most one
    // list, so they never meet); both are used last-in first-out.
    std::unique_ptr<int32_t[]> lists(new int32_t[m]);
    // p_i, the default entries and the lists, over row ranges in parallel:
    // each range counts its small rows first, so that it knows where its
    // share of either list starts, then fills it in index order.  A few
    // nanoseconds per row: threads pay for their start only from about 2^19
    // rows on.
    const unsigned parts = threads_for(m / 64);
    const int64_t chunk = (m + parts - 1) / parts;
    std::vector<int64_t> n_small(parts, 0);
    parallel_rows(m, parts, [&](int64_t lo, int64_t hi) {
        int64_t c = 0;
        for (int64_t i = lo; i < hi; ++i) {
            const double q = (w[i] * (double)m) / total;
            p[i] = q;
            c += q < 1.0;
            thresh[i] = 0xffffffffu;
            alias[i] = (int32_t)i;
        }
        n_small[lo / chunk] = c;
    });
    std::vector<int64_t> small_at(parts, 0);
    int64_t ns = 0;
    for (unsigned t = 0; t < parts; ++t) {
        small_at[t] = ns;
        ns += n_small[t];
    }
    int64_t nl = m - ns;
    parallel_rows(m, parts, [&](int64_t lo, int64_t hi) {
        int64_t sp = small_at[lo / chunk], lp = lo - sp;  // large rows before this range
        for (int64_t i = lo; i < hi; ++i) {
            if (p[i] < 1.0)
                lists[sp++] = (int32_t)i;
            else
                lists[m - 1 - lp++] = (int32_t)i;
        }
    });
    while (ns > 0 && nl > 0) {
        const int64_t sm = lists[--ns];
        const int64_t l = lists[m - nl--];
        thresh[sm] = (uint32_t)(uint64_t)(p[sm] * 4294967296.0);
        alias[sm] = (int32_t)l;
        p[l] = (p[l] + p[sm]) - 1.0;
        if (p[l] < 1.0)
            lists[ns++] = (int32_t)l;
        else
            lists[m - 1 - nl++] = (int32_t)l;
    }
    // leftovers keep thresh = 2^32 - 1 and alias = self
}

void build_alias(const std::vector<double> &w, std::vector<uint32_t> &thresh,
                 std::vector<int32_t> &alias) {
    double total = 0.0;
    for (double v : w) total = total + v;
    thresh.resize(w.size());
    alias.resize(w.size());
    build_alias(w.data(), (int64_t)w.size(), total, thresh.data(), alias.data());
}

void row_aux(const double *w, int64_t m, const uint32_t *thresh, const int32_t *alias, RowAux *aux) {
    parallel_rows(m, threads_for(m), [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) aux[i] = RowAux{1.0 / w[i], thresh[i], alias[i]};
    });
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

asyrk_status plan_records(int64_t m, const int64_t *row_ptr, int vk, SetupResult &res, int64_t *total_bytes) {
    const Geom g = geom_of(vk);
    auto raw_bytes = [&](int64_t nnz) { return (int64_t)g.HB + (nnz + g.U - 1) / g.U * g.UB; };
    int64_t total;
    if (res.fixed_nnz > 0) {
        res.stride = choose_stride(raw_bytes(res.fixed_nnz));
        res.loc.clear();
        total = res.stride * m;
    } else {
        res.stride = 0;
        res.loc.resize(m);
        int64_t off = 0;
        for (int64_t i = 0; i < m; ++i) {
            const int64_t nnz = row_ptr[i + 1] - row_ptr[i];
            if (off / 16 >= (int64_t)UINT32_MAX) return ASYRK_ERR_INVALID_ARG;
            res.loc[i] = RowLoc{(uint32_t)(off / 16), (uint32_t)nnz};
            off += raw_bytes(nnz);
        }
        total = off;
        if (total / 16 >= (int64_t)UINT32_MAX) return ASYRK_ERR_INVALID_ARG;
    }
    *total_bytes = total;
    return ASYRK_OK;
}

// Rows lo..hi-1 written in full: header, whole units, the last unit padded
// with (0, 0) entries, and (equal-length rows) zeros up to the stride.
template <int VK>
static void write_rows(int64_t lo, int64_t hi, const int64_t *row_ptr, const int32_t *col, const void *vals,
                       const double *b, const SetupResult &res, const uint32_t *thresh, const int32_t *alias,
                       uint8_t *dst) {
    using T = VT<VK>;
    using val_t = typename T::val_t;
    const val_t *vv = static_cast<const val_t *>(vals);
    const bool fixed = res.fixed_nnz > 0;
    for (int64_t i = lo; i < hi; ++i) {
        uint8_t *r = dst + (fixed ? i * res.stride : (int64_t)res.loc[i].off16 * 16);
        const double inv_w = 1.0 / res.w[i];
        if constexpr (VK == ASYRK_F64) {
            const HdrF64 h{b[i], inv_w, thresh[i], alias[i], 0};
            std::memcpy(r, &h, sizeof h);
        } else {
            const HdrF32 h{(float)b[i], (float)inv_w, thresh[i], alias[i]};
            std::memcpy(r, &h, sizeof h);
        }
        const int64_t beg = row_ptr[i], nnz = row_ptr[i + 1] - beg;
        const int32_t *c = col + beg;
        const val_t *v = vv + beg;
        uint8_t *u = r + T::HB;
        int64_t k = 0;
        for (; k + T::U <= nnz; k += T::U, u += T::UB) {
            std::memcpy(u, c + k, 4 * T::U);
            std::memcpy(u + T::COLB, v + k, T::VB * T::U);
        }
        if (k < nnz) {
            const int64_t rem = nnz - k;
            std::memset(u, 0, T::UB);
            std::memcpy(u, c + k, 4 * rem);
            std::memcpy(u + T::COLB, v + k, T::VB * rem);
            u += T::UB;
        }
        if (fixed) std::memset(u, 0, (size_t)(r + res.stride - u));
    }
}

void write_records(int64_t m, const int64_t *row_ptr, const int32_t *col, const void *vals, int vk,
                   const double *b, const SetupResult &res, const uint32_t *thresh, const int32_t *alias,
                   uint8_t *dst) {
    parallel_rows(m, threads_for(m), [&](int64_t lo, int64_t hi) {
        switch (vk) {
            case ASYRK_F64: write_rows<ASYRK_F64>(lo, hi, row_ptr, col, vals, b, res, thresh, alias, dst); break;
            case ASYRK_F32: write_rows<ASYRK_F32>(lo, hi, row_ptr, col, vals, b, res, thresh, alias, dst); break;
            default: write_rows<ASYRK_BF16>(lo, hi, row_ptr, col, vals, b, res, thresh, alias, dst); break;
        }
    });
}

asyrk_status pack_records(int64_t m, const int64_t *row_ptr, const int32_t *col, const void *vals,
                          int vk, const double *b, SetupResult &res) {
    const int64_t mm = (int64_t)res.w.size();
    std::unique_ptr<uint32_t[]> thresh(new uint32_t[mm]);
    std::unique_ptr<int32_t[]> alias(new int32_t[mm]);
    build_alias(res.w.data(), mm, res.fro2, thresh.get(), alias.get());
    int64_t total = 0;
    asyrk_status rc = plan_records(m, row_ptr, vk, res, &total);
    if (rc) return rc;
    try {
        res.rec.resize((size_t)total);
    } catch (...) {
        return ASYRK_ERR_OOM;
    }
    write_records(m, row_ptr, col, vals, vk, b, res, thresh.get(), alias.get(), res.rec.data());
    return ASYRK_OK;
}

}  // namespace asyrk
