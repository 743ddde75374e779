// Device-side building blocks of the sweep, shared by the single-system
// kernels (kernels.hip) and the packed serving kernels (server.hip).
#pragma once

#include <type_traits>

#include "internal.h"

namespace asyrk {

// ---------------------------------------------------------------- utilities

template <class T>
__device__ __forceinline__ T load_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float bf16_to_f32(uint32_t bits) { return __uint_as_float(bits << 16); }

__device__ __forceinline__ void locate(const Rows &r, uint32_t i, const uint8_t *&rec, int &nnz) {
    if (r.loc == nullptr) {
        rec = r.rec + (int64_t)i * r.stride;
        nnz = r.fixed_nnz;
    } else {
        const RowLoc l = r.loc[i];
        rec = r.rec + (int64_t)l.off16 * 16;
        nnz = (int)l.nnz;
    }
}

// 64 zero bytes: the read-only stand-in for an absent unit or row locator,
// so that loads can be issued unconditionally (no branch, no wait at a join).
static __device__ __attribute__((aligned(64))) const uint8_t kZeroPad[64] = {0};

// locate() without a branch: the locator is read from kZeroPad for
// fixed-stride rows and the values are picked by select.
__device__ __forceinline__ void locate_nb(const Rows &r, uint32_t i, const uint8_t *&rec, int &nnz) {
    const bool ragged = r.loc != nullptr;
    const RowLoc l = *(ragged ? r.loc + i : reinterpret_cast<const RowLoc *>(kZeroPad));
    rec = ragged ? r.rec + (int64_t)l.off16 * 16 : r.rec + (int64_t)i * r.stride;
    nnz = ragged ? (int)l.nnz : r.fixed_nnz;
}

template <int VK> struct Unit;
template <> struct Unit<ASYRK_F32> {
    int c[4];
    float v[4];
    __device__ __forceinline__ void load(const uint8_t *p) {
        const int4 ci = *reinterpret_cast<const int4 *>(p);
        const float4 vi = *reinterpret_cast<const float4 *>(p + 16);
        c[0] = ci.x; c[1] = ci.y; c[2] = ci.z; c[3] = ci.w;
        v[0] = vi.x; v[1] = vi.y; v[2] = vi.z; v[3] = vi.w;
    }
};
template <> struct Unit<ASYRK_BF16> {
    int c[8];
    float v[8];
    __device__ __forceinline__ void load(const uint8_t *p) {
        const int4 c0 = *reinterpret_cast<const int4 *>(p);
        const int4 c1 = *reinterpret_cast<const int4 *>(p + 16);
        const uint4 vb = *reinterpret_cast<const uint4 *>(p + 32);
        c[0] = c0.x; c[1] = c0.y; c[2] = c0.z; c[3] = c0.w;
        c[4] = c1.x; c[5] = c1.y; c[6] = c1.z; c[7] = c1.w;
        v[0] = bf16_to_f32(vb.x & 0xffffu); v[1] = bf16_to_f32(vb.x >> 16);
        v[2] = bf16_to_f32(vb.y & 0xffffu); v[3] = bf16_to_f32(vb.y >> 16);
        v[4] = bf16_to_f32(vb.z & 0xffffu); v[5] = bf16_to_f32(vb.z >> 16);
        v[6] = bf16_to_f32(vb.w & 0xffffu); v[7] = bf16_to_f32(vb.w >> 16);
    }
};
template <> struct Unit<ASYRK_F64> {
    int c[4];
    double v[4];
    __device__ __forceinline__ void load(const uint8_t *p) {
        const int4 ci = *reinterpret_cast<const int4 *>(p);
        const double2 v0 = *reinterpret_cast<const double2 *>(p + 16);
        const double2 v1 = *reinterpret_cast<const double2 *>(p + 32);
        c[0] = ci.x; c[1] = ci.y; c[2] = ci.z; c[3] = ci.w;
        v[0] = v0.x; v[1] = v0.y; v[2] = v1.x; v[3] = v1.y;
    }
};

template <int VK>
__device__ __forceinline__ typename VT<VK>::hdr_t load_hdr(const uint8_t *rec) {
    return *reinterpret_cast<const typename VT<VK>::hdr_t *>(rec);
}

// Entry `pos` of a row record (column, value), read directly.
template <int VK>
__device__ __forceinline__ void load_entry(const uint8_t *rec, int pos, int &c,
                                           typename VT<VK>::x_t &v) {
    using T = VT<VK>;
    const uint8_t *u = rec + T::HB + (int64_t)(pos / T::U) * T::UB;
    const int e = pos % T::U;
    c = *reinterpret_cast<const int *>(u + 4 * e);
    if constexpr (VK == ASYRK_BF16)
        v = bf16_to_f32(*reinterpret_cast<const uint16_t *>(u + T::COLB + 2 * e));
    else
        v = *reinterpret_cast<const typename T::val_t *>(u + T::COLB + T::VB * e);
}

template <int G, class X>
__device__ __forceinline__ X group_sum(X v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Units per lane kept in registers: a row of up to G * UPL units is read
// once; longer rows are read twice (dot pass, then scatter pass).
template <int G> struct Upl { static constexpr int value = G >= 8 ? 1 : 8 / G; };

// ---------------------------------------------------------------- sweep

// One ticket of one worker (a group of G lanes): draw the row, fetch its
// record, gather-dot, step, atomic scatter.  XK: iterate dtype.  FP32 records
// with an FP64 iterate read b_i and 1/w_i in FP64 from the side array (the
// record header holds them in FP32).  Returns the read-to-write window in
// clock ticks when `trace` is set.
// Row i of a sweep given directly (no sampling): used by the slice scheme.
// `alias_ok` = false keeps row i whatever its header says.
template <int VK, int XK, int G, int UPL = Upl<G>::value, bool SAMPLED = true>
__device__ __forceinline__ uint64_t process_ticket(
    const Rows &rows, typename std::conditional<XK == ASYRK_F64, double, float>::type *x,
    const double2 *side, int64_t j, uint32_t stream_id, uint32_t k0, uint32_t k1, int uniform,
    int update_one, typename std::conditional<XK == ASYRK_F64, double, float>::type gamma, int gl,
    int trace, uint32_t given_row = 0) {
    using T = VT<VK>;
    using X = typename std::conditional<XK == ASYRK_F64, double, float>::type;
    using H = typename T::hdr_t;
    constexpr bool SIDE = (XK == ASYRK_F64) && (VK != ASYRK_F64);
    constexpr int U = T::U;

    // a1: ticket -> bucket -> row (alias decision needs the header); or a given row
    U4 u{0u, 0u, 0u, 0u};
    uint32_t i = given_row;
    if constexpr (SAMPLED) {
        u = draw(j, stream_id, k0, k1);
        i = bucket_of(u.a, u.b, (uint32_t)rows.m);
    }
    const uint8_t *rec;
    int nnz;
    locate(rows, i, rec, nnz);
    H h = load_hdr<VK>(rec);
    int nunits = (nnz + U - 1) / U;
    // a2: speculative fetch of the bucket row's units (the alias is rarely taken)
    Unit<VK> un[UPL];
#pragma unroll
    for (int q = 0; q < UPL; ++q) {
        const int uu = gl + q * G;
        if (uu < nunits) un[q].load(rec + T::HB + (int64_t)uu * T::UB);
    }
    if (SAMPLED && !uniform && !(u.c < h.thresh)) {
        i = (uint32_t)h.alias;
        locate(rows, i, rec, nnz);
        h = load_hdr<VK>(rec);
        nunits = (nnz + U - 1) / U;
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int uu = gl + q * G;
            if (uu < nunits) un[q].load(rec + T::HB + (int64_t)uu * T::UB);
        }
    }

    uint64_t t0 = 0;
    if (trace) t0 = wall_clock64();

    // a3: gather-dot over supp(a_i)
    X acc = (X)0;
    const bool one_pass = nunits <= G * UPL;
    if (one_pass) {
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int uu = gl + q * G;
            if (uu < nunits) {
#pragma unroll
                for (int e = 0; e < U; ++e) {
                    if (uu * U + e < nnz) acc = fma((X)un[q].v[e], load_agent(x + un[q].c[e]), acc);
                }
            }
        }
    } else {
        for (int base = 0; base < nunits; base += G * UPL) {
            if (base > 0) {
#pragma unroll
                for (int q = 0; q < UPL; ++q) {
                    const int uu = base + gl + q * G;
                    if (uu < nunits) un[q].load(rec + T::HB + (int64_t)uu * T::UB);
                }
            }
#pragma unroll
            for (int q = 0; q < UPL; ++q) {
                const int uu = base + gl + q * G;
                if (uu < nunits) {
#pragma unroll
                    for (int e = 0; e < U; ++e)
                        if (uu * U + e < nnz) acc = fma((X)un[q].v[e], load_agent(x + un[q].c[e]), acc);
                }
            }
        }
    }
    acc = group_sum<G>(acc);

    // a4: step s = gamma * (a_i^T x - b_i) / ||a_i||^2
    X bi, inv_w;
    if constexpr (SIDE) {
        const double2 sd = side[i];
        bi = sd.x;
        inv_w = sd.y;
    } else {
        bi = (X)h.b;
        inv_w = (X)h.inv_w;
    }
    const X r = acc - bi;

    // a5: lock-free scatter
    if (!update_one) {
        const X s = gamma * r * inv_w;
        if (one_pass) {
#pragma unroll
            for (int q = 0; q < UPL; ++q) {
                const int uu = gl + q * G;
                if (uu < nunits) {
#pragma unroll
                    for (int e = 0; e < U; ++e)
                        if (uu * U + e < nnz) unsafeAtomicAdd(x + un[q].c[e], -s * (X)un[q].v[e]);
                }
            }
        } else {
            for (int base = 0; base < nunits; base += G * UPL) {
#pragma unroll
                for (int q = 0; q < UPL; ++q) {
                    const int uu = base + gl + q * G;
                    if (uu < nunits) {
                        un[q].load(rec + T::HB + (int64_t)uu * T::UB);
#pragma unroll
                        for (int e = 0; e < U; ++e)
                            if (uu * U + e < nnz) unsafeAtomicAdd(x + un[q].c[e], -s * (X)un[q].v[e]);
                    }
                }
            }
        }
    } else if (gl == 0) {
        // Algorithm 1: one coordinate t, step gamma * theta_i
        const int t = (int)(((uint64_t)u.d * (uint64_t)nnz) >> 32);
        int c;
        typename VT<VK>::x_t v;
        load_entry<VK>(rec, t, c, v);
        const X s1 = gamma * (X)nnz * r * inv_w;
        unsafeAtomicAdd(x + c, -s1 * (X)v);
    }
    return trace ? wall_clock64() - t0 : 0;
}

// The tickets j0, j0 + step, ... < j_end of one worker with the steps of
// process_ticket (sampled rows, all-coordinate update), arranged so that a
// ticket costs two dependent memory round trips instead of one per access:
//
//   1. the next ticket's row locator is requested together with this
//      ticket's gathers, which are issued back to back (padded slots read
//      x[0] and are masked out by a select, so no branch splits them) and
//      waited for once;
//   2. the atomics are issued while no load is outstanding, then the next
//      ticket's record is requested; its wait overlaps the atomics.
//
// Row records are read-only during a sweep, so fetching the next record
// early moves no read of x: the gathers of ticket t + 1 are still issued
// after the atomics of ticket t.
template <int VK, int XK, int G, int UPL = Upl<G>::value>
__device__ __forceinline__ void run_tickets_pipelined(
    const Rows rows, typename std::conditional<XK == ASYRK_F64, double, float>::type *x,
    const double2 *side, int64_t j, int64_t j_end, int64_t step, uint32_t stream_id, uint32_t k0,
    uint32_t k1, int uniform, typename std::conditional<XK == ASYRK_F64, double, float>::type gamma,
    int gl) {
    using T = VT<VK>;
    using X = typename std::conditional<XK == ASYRK_F64, double, float>::type;
    using H = typename T::hdr_t;
    constexpr bool SIDE = (XK == ASYRK_F64) && (VK != ASYRK_F64);
    constexpr int U = T::U;
    if (j >= j_end) return;

    // units base + gl, base + gl + G, ... of a row; absent units are read
    // from kZeroPad, so every load is issued unconditionally
    static_assert(T::UB <= (int)sizeof(kZeroPad), "zero pad smaller than a unit");
    auto fetch_chunk = [&](const uint8_t *rec, int base, int nunits, Unit<VK> *dst) {
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int uu = base + gl + q * G;
            dst[q].load(uu < nunits ? rec + T::HB + (int64_t)uu * T::UB : kZeroPad);
        }
    };
    auto fetch_units = [&](const uint8_t *rec, int nunits, Unit<VK> *dst) { fetch_chunk(rec, 0, nunits, dst); };
    // branch-free gather-dot of one chunk held in registers
    auto chunk_dot = [&](const Unit<VK> *cu, int base, int nnz, X acc) {
        X xv[UPL][U];
#pragma unroll
        for (int q = 0; q < UPL; ++q)
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const bool ok = (base + gl + q * G) * U + e < nnz;
                xv[q][e] = load_agent(x + (ok ? cu[q].c[e] : 0));
            }
#pragma unroll
        for (int q = 0; q < UPL; ++q)
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const bool ok = (base + gl + q * G) * U + e < nnz;
                acc = ok ? fma((X)cu[q].v[e], xv[q][e], acc) : acc;
            }
        return acc;
    };
    auto chunk_scatter = [&](const Unit<VK> *cu, int base, int nnz, X s) {
#pragma unroll
        for (int q = 0; q < UPL; ++q)
#pragma unroll
            for (int e = 0; e < U; ++e)
                if ((base + gl + q * G) * U + e < nnz) unsafeAtomicAdd(x + cu[q].c[e], -s * (X)cu[q].v[e]);
    };
    // the alias branch of the draw (needs the bucket row's header)
    auto resolve = [&](const U4 &u, uint32_t &i, const uint8_t *&rec, int &nnz, H &h, Unit<VK> *dst) {
        if (!uniform && !(u.c < h.thresh)) {
            i = (uint32_t)h.alias;
            locate_nb(rows, i, rec, nnz);
            h = load_hdr<VK>(rec);
            fetch_units(rec, (nnz + U - 1) / U, dst);
        }
    };
    auto coeffs = [&](uint32_t i, const H &h, X &bi, X &inv_w) {
        if constexpr (SIDE) {
            const double2 sd = side[i];
            bi = sd.x;
            inv_w = sd.y;
        } else {
            bi = (X)h.b;
            inv_w = (X)h.inv_w;
        }
    };

    // prologue: the first ticket, fetched in full
    U4 u = draw(j, stream_id, k0, k1);
    uint32_t i = bucket_of(u.a, u.b, (uint32_t)rows.m);
    const uint8_t *rec;
    int nnz;
    locate_nb(rows, i, rec, nnz);
    H h = load_hdr<VK>(rec);
    Unit<VK> un[UPL];
    fetch_units(rec, (nnz + U - 1) / U, un);
    resolve(u, i, rec, nnz, h, un);
    X bi, inv_w;
    coeffs(i, h, bi, inv_w);

    for (;;) {
        const int64_t jn = j + step;
        const bool more = jn < j_end;
        // the next ticket's row and locator, requested with this ticket's gathers
        // (drawn even past the end: the row is valid and simply not used)
        U4 u2 = draw(jn, stream_id, k0, k1);
        uint32_t i2 = bucket_of(u2.a, u2.b, (uint32_t)rows.m);
        const uint8_t *rec2;
        int nnz2;
        locate_nb(rows, i2, rec2, nnz2);
        // gather-dot: first chunk from registers, further chunks (long rows) re-read
        const int nunits = (nnz + U - 1) / U;
        X acc = chunk_dot(un, 0, nnz, (X)0);
        for (int base = G * UPL; base < nunits; base += G * UPL) {
            Unit<VK> t[UPL];
            fetch_chunk(rec, base, nunits, t);
            acc = chunk_dot(t, base, nnz, acc);
        }
        acc = group_sum<G>(acc);
        const X s = gamma * (acc - bi) * inv_w;
        // lock-free scatter
        chunk_scatter(un, 0, nnz, s);
        for (int base = G * UPL; base < nunits; base += G * UPL) {
            Unit<VK> t[UPL];
            fetch_chunk(rec, base, nunits, t);
            chunk_scatter(t, base, nnz, s);
        }
        if (!more) break;
        // the next ticket's record; its wait overlaps the atomics above
        H h2 = load_hdr<VK>(rec2);
        Unit<VK> un2[UPL];
        fetch_units(rec2, (nnz2 + U - 1) / U, un2);
        resolve(u2, i2, rec2, nnz2, h2, un2);
        coeffs(i2, h2, bi, inv_w);
        j = jn;
        u = u2;
        i = i2;
        rec = rec2;
        nnz = nnz2;
        h = h2;
#pragma unroll
        for (int q = 0; q < UPL; ++q) un[q] = un2[q];
    }
}

// Keyed bijection of [0, L) for the slice scheme: with b the smallest width
// such that 2^b >= L, mask = 2^b - 1 and h = (b + 1) / 2, apply
//   y <- ((y ^ (y >> h)) * (u0 | 1) + u1) & mask
//   y <- ((y ^ (y >> h)) * (u2 | 1) + u3) & mask
// (each step is a bijection of [0, 2^b)) until y < L (cycle walking).
// (u0..u3) = Philox4x32-10(counter (sweep lo, sweep hi, worker, 0x5C4E3D2B), key = seed).
__device__ __forceinline__ uint32_t slice_perm(uint32_t k, uint32_t L, const U4 &u) {
    if (L <= 1) return 0;
    const uint32_t b = 32 - __clz(L - 1);
    const uint32_t mask = b >= 32 ? 0xffffffffu : ((1u << b) - 1u);
    const uint32_t h = (b + 1) / 2;
    uint32_t y = k;
    do {
        y = ((y ^ (y >> h)) * (u.a | 1u) + u.b) & mask;
        y = ((y ^ (y >> h)) * (u.c | 1u) + u.d) & mask;
    } while (y >= L);
    return y;
}

}  // namespace asyrk
