// Host setup code (CSR validation, row weights, alias table, record packing,
// augmented system) run under AddressSanitizer and UBSan: valid systems of
// every value dtype and layout, then invalid inputs, each of which must be
// rejected with its documented status.  Exit status 0 = every check held.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "setup.h"

using namespace asyrk;

static int g_fail = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++g_fail;                                                    \
        }                                                                \
    } while (0)

struct Sys {
    int64_t m = 0, n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<double> v64;
    std::vector<float> v32;
    std::vector<uint16_t> v16;
    std::vector<double> b;
    const void *vals(int vk) const {
        return vk == ASYRK_F64 ? (const void *)v64.data()
                               : vk == ASYRK_F32 ? (const void *)v32.data() : (const void *)v16.data();
    }
};

static uint16_t to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// rows of lo..hi distinct sorted columns (lo >= 1), N(0,1) values
static Sys make(std::mt19937_64 &g, int64_t m, int64_t n, int lo, int hi) {
    Sys s;
    s.m = m;
    s.n = n;
    s.rp.push_back(0);
    std::normal_distribution<double> nd;
    for (int64_t i = 0; i < m; ++i) {
        const int64_t want = std::min<int64_t>(n, lo + (int64_t)(g() % (uint64_t)(hi - lo + 1)));
        std::vector<int32_t> cs;
        while ((int64_t)cs.size() < want) {
            const int32_t c = (int32_t)(g() % (uint64_t)n);
            bool seen = false;
            for (int32_t q : cs) seen |= q == c;
            if (!seen) cs.push_back(c);
        }
        std::sort(cs.begin(), cs.end());
        for (int32_t c : cs) {
            s.col.push_back(c);
            const double v = nd(g);
            s.v64.push_back(v);
            s.v32.push_back((float)v);
            s.v16.push_back(to_bf16((float)v));
        }
        s.rp.push_back((int64_t)s.col.size());
        s.b.push_back(nd(g));
    }
    return s;
}

int main() {
    std::mt19937_64 g(12345);
    const int vks[3] = {ASYRK_F64, ASYRK_F32, ASYRK_BF16};
    for (int trial = 0; trial < 24; ++trial) {
        const int64_t m = 1 + (int64_t)(g() % 300), n = 1 + (int64_t)(g() % 200);
        const bool fixed = trial % 3 == 0;
        const int lo = fixed ? 7 : 1, hi = fixed ? 7 : 70;
        Sys s = make(g, m, n, lo, hi);
        for (int vk : vks) {
            SetupResult r;
            CHECK(validate_system(m, n, s.rp.data(), s.col.data(), s.vals(vk), vk, s.b.data(), r) == ASYRK_OK);
            CHECK(pack_records(m, s.rp.data(), s.col.data(), s.vals(vk), vk, s.b.data(), r) == ASYRK_OK);
            CHECK(!r.rec.empty());
            CHECK(r.fixed_nnz > 0 || (int64_t)r.loc.size() == m);
            std::vector<uint32_t> t;
            std::vector<int32_t> al;
            build_alias(r.w, t, al);
            CHECK((int64_t)t.size() == m && (int64_t)al.size() == m);
            for (int64_t i = 0; i < m; ++i) CHECK(al[i] >= 0 && al[i] < m);
            // an empty column of A is an all-zero row of the augmented matrix
            std::vector<int> used(n, 0);
            for (int32_t c : s.col) used[c] = 1;
            const bool full = std::find(used.begin(), used.end(), 0) == used.end();
            AugCSR aug;
            const asyrk_status ra =
                build_augmented(m, n, s.rp.data(), s.col.data(), s.vals(vk), vk, s.b.data(), 0.5, 1.0, aug);
            CHECK(ra == (full ? ASYRK_OK : ASYRK_ERR_ZERO_ROW));
            if (full) CHECK((int64_t)aug.row_ptr.size() == m + n + 1);
            AugCSR bad;
            CHECK(build_augmented(m, n, s.rp.data(), s.col.data(), s.vals(vk), vk, s.b.data(), 0.0, 1.0, bad) ==
                  ASYRK_ERR_INVALID_ARG);
        }
    }
    // systems large enough for the threaded validation and record writing
    // (one host thread per 4096 rows), valid and with invalid entries that
    // the concurrent column pass must not follow out of range
    for (int trial = 0; trial < 3; ++trial) {
        const int64_t m = 20000 + 4000 * trial, n = 3000;
        Sys big = make(g, m, n, 1, 40);
        for (int vk : vks) {
            SetupResult r;
            CHECK(validate_system(m, n, big.rp.data(), big.col.data(), big.vals(vk), vk, big.b.data(), r) == ASYRK_OK);
            CHECK(pack_records(m, big.rp.data(), big.col.data(), big.vals(vk), vk, big.b.data(), r) == ASYRK_OK);
            CHECK(r.nnz == big.rp[m] && r.nu >= 1 && r.mu >= 1 && r.max_col_norm2 > 0.0);
        }
        for (int bad = 0; bad < 3; ++bad) {
            Sys q = big;
            const int64_t k = q.rp[m / 2 + bad];
            if (bad == 0) q.col[k] = (int32_t)n + 5;      // out of range
            if (bad == 1) q.col[k] = -7;                  // negative
            if (bad == 2) q.v64[k] = std::nan("");        // not finite
            SetupResult rr;
            CHECK(validate_system(m, n, q.rp.data(), q.col.data(), q.vals(ASYRK_F64), ASYRK_F64, q.b.data(), rr) ==
                  ASYRK_ERR_INVALID_ARG);
        }
    }
    // the alias table's classification pass runs over row ranges in parallel
    // from about 2^19 rows on: the table must equal the sequential
    // construction's (written out here from its definition), entry for entry
    {
        const int64_t m = 600000;
        std::vector<double> w(m);
        std::lognormal_distribution<double> ln(0.0, 1.5);
        for (auto &x : w) x = ln(g);
        std::vector<uint32_t> t;
        std::vector<int32_t> al;
        build_alias(w, t, al);
        double total = 0.0;
        for (double x : w) total = total + x;
        std::vector<double> p(m);
        std::vector<int32_t> small, large;
        for (int64_t i = 0; i < m; ++i) {
            p[i] = (w[i] * (double)m) / total;
            (p[i] < 1.0 ? small : large).push_back((int32_t)i);
        }
        std::vector<uint32_t> t2(m, 0xffffffffu);
        std::vector<int32_t> a2(m);
        for (int64_t i = 0; i < m; ++i) a2[i] = (int32_t)i;
        while (!small.empty() && !large.empty()) {
            const int32_t sm = small.back();
            small.pop_back();
            const int32_t l = large.back();
            large.pop_back();
            t2[sm] = (uint32_t)(uint64_t)(p[sm] * 4294967296.0);
            a2[sm] = l;
            p[l] = (p[l] + p[sm]) - 1.0;
            (p[l] < 1.0 ? small : large).push_back(l);
        }
        CHECK(t == t2);
        CHECK(al == a2);
    }
    // invalid inputs
    Sys s = make(g, 50, 40, 2, 6);
    SetupResult r;
    const int vk = ASYRK_F64;
    auto val = [&](Sys &q) {
        SetupResult rr;
        return validate_system(q.m, q.n, q.rp.data(), q.col.data(), q.vals(vk), vk, q.b.data(), rr);
    };
    {
        Sys q = s;
        std::swap(q.col[q.rp[3]], q.col[q.rp[3] + 1]);  // unsorted
        CHECK(val(q) == ASYRK_ERR_INVALID_ARG);
    }
    {
        Sys q = s;
        q.col[q.rp[4] + 1] = q.col[q.rp[4]];  // duplicate
        CHECK(val(q) == ASYRK_ERR_INVALID_ARG);
    }
    {
        Sys q = s;
        q.col[q.rp[5 + 1] - 1] = (int32_t)q.n;  // out of range
        CHECK(val(q) == ASYRK_ERR_INVALID_ARG);
    }
    {
        Sys q = s;
        q.col[q.rp[6]] = -3;  // negative
        CHECK(val(q) == ASYRK_ERR_INVALID_ARG);
    }
    {
        Sys q = s;
        q.v64[q.rp[7]] = std::nan("");
        CHECK(val(q) == ASYRK_ERR_INVALID_ARG);
    }
    {
        Sys q = s;
        q.b[9] = INFINITY;
        CHECK(val(q) == ASYRK_ERR_INVALID_ARG);
    }
    {
        Sys q = s;
        for (int64_t k = q.rp[10]; k < q.rp[11]; ++k) q.v64[k] = 0.0;  // zero row
        CHECK(val(q) == ASYRK_ERR_ZERO_ROW);
    }
    {
        Sys q = s;
        q.rp[12] = q.rp[13] + 1;  // decreasing row pointer
        CHECK(val(q) == ASYRK_ERR_INVALID_ARG);
    }
    {
        Sys q = s;
        q.rp[0] = 1;
        CHECK(val(q) == ASYRK_ERR_INVALID_ARG);
    }
    CHECK(validate_system(0, 4, s.rp.data(), s.col.data(), s.v64.data(), vk, s.b.data(), r) == ASYRK_ERR_INVALID_ARG);
    CHECK(validate_system(s.m, s.n, s.rp.data(), s.col.data(), s.v64.data(), 7, s.b.data(), r) ==
          ASYRK_ERR_INVALID_ARG);
    std::printf("setup sanitizer run: %d failed checks\n", g_fail);
    return g_fail ? 1 : 0;
}
