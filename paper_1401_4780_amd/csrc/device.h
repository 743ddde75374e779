// Device-side building blocks of the sweep, shared by the single-system
// kernels (kernels.hip) and the packed serving kernels (server.hip).
#pragma once

#include <cstddef>
#include <type_traits>

#include "internal.h"

namespace asyrk {

// ---------------------------------------------------------------- utilities

// Every pointer the sweep dereferences is device global memory (records,
// locators, side records, the iterate, the zero pad).  Saying so turns the
// generic (flat) accesses the compiler emits for pointers it cannot trace -
// loaded from a table, or selected between two arrays - into global ones:
// flat accesses may complete out of order with other memory accesses, so
// while one is outstanding every wait becomes a wait for everything.
#define ASYRK_GLOBAL __attribute__((address_space(1)))

typedef uint32_t gv2u __attribute__((ext_vector_type(2)));
typedef uint32_t gv4u __attribute__((ext_vector_type(4)));

// A load of T from global memory.  Structs (int4, float4, headers, locators)
// are read as native vectors of the same size and copied bitwise: copying a
// struct through its copy constructor would read it through a generic
// reference and bring the flat access back.  T must be naturally aligned.
template <class T>
__device__ __forceinline__ T gload(const void *p) {
    T out;
    if constexpr (sizeof(T) == 2) {
        const uint16_t v = *(const ASYRK_GLOBAL uint16_t *)p;
        __builtin_memcpy(&out, &v, 2);
    } else if constexpr (sizeof(T) == 4) {
        const uint32_t v = *(const ASYRK_GLOBAL uint32_t *)p;
        __builtin_memcpy(&out, &v, 4);
    } else if constexpr (sizeof(T) == 8) {
        const gv2u v = *(const ASYRK_GLOBAL gv2u *)p;
        __builtin_memcpy(&out, &v, 8);
    } else if constexpr (sizeof(T) == 16) {
        const gv4u v = *(const ASYRK_GLOBAL gv4u *)p;
        __builtin_memcpy(&out, &v, 16);
    } else {
        static_assert(sizeof(T) == 32, "gload: unsupported size");
        const gv4u a = *(const ASYRK_GLOBAL gv4u *)p;
        const gv4u b = *(const ASYRK_GLOBAL gv4u *)((const uint8_t *)p + 16);
        __builtin_memcpy(&out, &a, 16);
        __builtin_memcpy(reinterpret_cast<uint8_t *>(&out) + 16, &b, 16);
    }
    return out;
}

template <class T>
__device__ __forceinline__ T load_agent(const T *p) {
    return __hip_atomic_load((const ASYRK_GLOBAL T *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// no-return atomic add at agent scope (a hardware float atomic)
template <class T>
__device__ __forceinline__ void atomic_add(T *p, T v) {
    (void)__hip_atomic_fetch_add((ASYRK_GLOBAL T *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Element c of an iterate stored with a stride of 2^sh elements: columns that
// would share a cache line get lines of their own, so their gathers and
// atomics do not queue behind each other.
template <class T>
__device__ __forceinline__ T *xat(T *x, int32_t c, int sh) {
    return x + ((int64_t)c << sh);
}

__device__ __forceinline__ float bf16_to_f32(uint32_t bits) { return __uint_as_float(bits << 16); }

__device__ __forceinline__ void locate(const Rows &r, uint32_t i, const uint8_t *&rec, int &nnz) {
    if (r.loc == nullptr) {
        rec = r.rec + (int64_t)i * r.stride;
        nnz = r.fixed_nnz;
    } else {
        const RowLoc l = gload<RowLoc>(r.loc + i);
        rec = r.rec + (int64_t)l.off16 * 16;
        nnz = (int)l.nnz;
    }
}

// 64 zero bytes: the stand-in for an absent unit or row locator, so that
// loads can be issued unconditionally (no branch, no wait at a join).  Never
// written.  Not declared const: a const device array lives in the constant
// address space, and a pointer selected between it and a global array can
// only be generic, which brings back the flat accesses avoided above.
static __device__ __attribute__((aligned(64))) uint8_t kZeroPad[64] = {0};

// locate() without a branch: the locator is read from kZeroPad for
// fixed-stride rows and the values are picked by select.
__device__ __forceinline__ void locate_nb(const Rows &r, uint32_t i, const uint8_t *&rec, int &nnz) {
    const bool ragged = r.loc != nullptr;
    const RowLoc l = gload<RowLoc>(ragged ? (const void *)(r.loc + i) : (const void *)kZeroPad);
    rec = ragged ? r.rec + (int64_t)l.off16 * 16 : r.rec + (int64_t)i * r.stride;
    nnz = ragged ? (int)l.nnz : r.fixed_nnz;
}

template <int VK> struct Unit;
template <> struct Unit<ASYRK_F32> {
    int c[4];
    float v[4];
    __device__ __forceinline__ void load(const uint8_t *p) {
        const int4 ci = gload<int4>(p);
        const float4 vi = gload<float4>(p + 16);
        c[0] = ci.x; c[1] = ci.y; c[2] = ci.z; c[3] = ci.w;
        v[0] = vi.x; v[1] = vi.y; v[2] = vi.z; v[3] = vi.w;
    }
};
template <> struct Unit<ASYRK_BF16> {
    int c[8];
    float v[8];
    __device__ __forceinline__ void load(const uint8_t *p) {
        const int4 c0 = gload<int4>(p);
        const int4 c1 = gload<int4>(p + 16);
        const uint4 vb = gload<uint4>(p + 32);
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
        const int4 ci = gload<int4>(p);
        const double2 v0 = gload<double2>(p + 16);
        const double2 v1 = gload<double2>(p + 32);
        c[0] = ci.x; c[1] = ci.y; c[2] = ci.z; c[3] = ci.w;
        v[0] = v0.x; v[1] = v0.y; v[2] = v1.x; v[3] = v1.y;
    }
};

template <int VK>
__device__ __forceinline__ typename VT<VK>::hdr_t load_hdr(const uint8_t *rec) {
    return gload<typename VT<VK>::hdr_t>(rec);
}

// Entry `pos` of a row record (column, value), read directly.
template <int VK>
__device__ __forceinline__ void load_entry(const uint8_t *rec, int pos, int &c,
                                           typename VT<VK>::x_t &v) {
    using T = VT<VK>;
    const uint8_t *u = rec + T::HB + (int64_t)(pos / T::U) * T::UB;
    const int e = pos % T::U;
    c = gload<int>(u + 4 * e);
    if constexpr (VK == ASYRK_BF16)
        v = bf16_to_f32(gload<uint16_t>(u + T::COLB + 2 * e));
    else
        v = gload<typename T::val_t>(u + T::COLB + T::VB * e);
}

// ---------------------------------------------------------------- staleness
//
// The delay of eq. (3), measured: for a sampled ticket, the number of row
// updates other waves completed between its read of x and its scatter
// (j - k(j) in the paper's notation).  A completion counter is split over
// kTauShards words, each on a line of its own.  Every worker counts its rows;
// every kTauFlush steps a wave adds the rows its workers finished since the
// last add to its shard (one atomic per wave per kTauFlush steps, after the
// scatter), and a worker that runs out of tickets adds what it has left.
// On steps kTauFlush, kTauFlush + kTauPeriod, ... of a launch (the first
// after every wave has added once) a wave reads the counter (the sum of the
// shards) just before its gathers and again just before it issues its
// scatter, so a lone worker measures exactly 0.  The reads are agent-scope atomic loads and
// the adds agent-scope atomics on the same words, so a wave's later read sees
// its own earlier adds.  Rows of other waves finished in the window but not
// yet added are missed and rows finished earlier but added in the window are
// counted: each sample is exact up to that backlog (at most kTauFlush steps
// of each wave), and unbiased on average.  The workers of one wave step
// together, so each also runs concurrently with up to 64/G - 1 updates of its
// own wave that the counter does not include.
constexpr int kTauShards = 16;
constexpr int kTauShardStride = 32;  // u64 words between shards (256 B)
constexpr int kTauPeriod = 64;       // steps between samples of one wave
constexpr int kTauFlush = 4;         // steps between a wave's adds
constexpr int kTraceWords = 8;       // per wave: {tau max, tau sum, samples, window max, window sum, 0, 0, 0}

struct TauProbe {
    const uint64_t *ctr;  // counter shards
    bool sample;          // read the counter around this ticket
    uint64_t c0, c1;      // counter before the gathers, before the scatter
    uint64_t t0, t1;      // wall clock at those points
};

// per-wave accumulators (identical in every lane: the counter reads of one
// instruction return one value to all lanes)
struct TauAcc {
    uint64_t tmax = 0, tsum = 0, tcnt = 0, wmax = 0, wsum = 0;
};

// The counter: every lane loads every shard (one address per instruction).
__device__ __forceinline__ uint64_t tau_read(const uint64_t *ctr) {
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kTauShards; ++k) s += load_agent(ctr + k * kTauShardStride);
    return s;
}

// The same read in two halves: the loads, and later their sum (so that the
// wave need not wait for them where they are issued).
__device__ __forceinline__ void tau_issue(const uint64_t *ctr, uint64_t (&v)[kTauShards]) {
#pragma unroll
    for (int k = 0; k < kTauShards; ++k) v[k] = load_agent(ctr + k * kTauShardStride);
}
__device__ __forceinline__ uint64_t tau_sum(const uint64_t (&v)[kTauShards]) {
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kTauShards; ++k) s += v[k];
    return s;
}

__device__ __forceinline__ void tau_accumulate(TauAcc &acc, uint64_t c0, uint64_t c1, uint64_t t0, uint64_t t1) {
    const uint64_t d = c1 - c0;  // each shard is read later at c1 than at c0: c1 >= c0
    const uint64_t w = t1 - t0;
    acc.tmax = d > acc.tmax ? d : acc.tmax;
    acc.tsum += d;
    acc.tcnt += 1;
    acc.wmax = w > acc.wmax ? w : acc.wmax;
    acc.wsum += w;
}

// A wave's add: the rows `mine` (< 8) its active group leaders finished since
// their last add, summed bit by bit over ballots, added by the lowest active
// lane to the wave's shard; every leader's count is then cleared.
__device__ __forceinline__ void tau_flush_wave(uint64_t *ctr, int64_t wave, int gl, uint32_t &mine) {
    const bool lead = gl == 0;
    uint64_t total = 0;
#pragma unroll
    for (int bit = 0; bit < 3; ++bit)
        total += (uint64_t)__popcll(__ballot(lead && ((mine >> bit) & 1u))) << bit;
    const unsigned long long active = __ballot(1);
    if ((int)__lane_id() == __ffsll(active) - 1 && total > 0)
        atomic_add(ctr + (wave & (kTauShards - 1)) * kTauShardStride, total);
    mine = 0;
}

// A leader's own remainder when it leaves the loop.
__device__ __forceinline__ void tau_flush_leader(uint64_t *ctr, int64_t wave, int gl, uint32_t &mine) {
    if (gl == 0 && mine > 0) atomic_add(ctr + (wave & (kTauShards - 1)) * kTauShardStride, (uint64_t)mine);
    mine = 0;
}

__device__ __forceinline__ void tau_store(const TauAcc &acc, uint64_t *out, int64_t wave, int lane) {
    if (lane == 0) {
        uint64_t *o = out + wave * kTraceWords;
        o[0] = acc.tmax;
        o[1] = acc.tsum;
        o[2] = acc.tcnt;
        o[3] = acc.wmax;
        o[4] = acc.wsum;
    }
}

// One DPP lane move of a 32- or 64-bit value (a 64-bit value moves as its
// two halves).  ROWS = 0xF: a pattern that gives every lane a source in its
// own row (quad permutations, mirrors), so every lane is written.  Otherwise
// the lanes of the rows outside the mask read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_move32(int v) {
    if constexpr (ROWS == 0xF) return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
    else return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, dpp_move32<CTRL, ROWS>(__builtin_bit_cast(int, v)));
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_move(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)dpp_move32<CTRL, ROWS>((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)dpp_move32<CTRL, ROWS>((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <class X>
__device__ __forceinline__ X read_lane(X v, int lane) {
    if constexpr (sizeof(X) == 8) {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
        return __builtin_bit_cast(X, ((uint64_t)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(X, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
    }
}

// Sum over each aligned group of G lanes, returned to every lane of the group.
// Within a 16-lane row the moves are register-to-register DPP (quad
// permutations, then the half-row and row mirrors: after each step the value
// is uniform over the lanes summed so far, so a mirror adds the other half's
// sum).  Across rows, row_bcast15 adds row 0 into row 1 and row 2 into row 3,
// row_bcast31 adds rows 0 + 1 into rows 2 and 3, and the group's total is read
// from its last lane.  No LDS traffic, so no wait on the LDS counter; every
// lane of a group ends with the same bits.  The lanes of a group must be
// active together (a group is one worker).
template <int G, class X>
__device__ __forceinline__ X group_sum(X v) {
    if constexpr (G >= 2) v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
    if constexpr (G >= 4) v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
    if constexpr (G >= 8) v += dpp_move<0x141>(v);  // row_half_mirror
    if constexpr (G >= 16) v += dpp_move<0x140>(v); // row_mirror
    if constexpr (G == 32) {
        v += dpp_move<0x142, 0xA>(v);                // row_bcast15 into rows 1, 3
        const X lo = read_lane(v, 31), hi = read_lane(v, 63);
        v = (__lane_id() < 32) ? lo : hi;
    } else if constexpr (G == 64) {
        v += dpp_move<0x142, 0xA>(v);                // row_bcast15 into rows 1, 3
        v += dpp_move<0x143, 0xC>(v);                // row_bcast31 into rows 2, 3
        v = read_lane(v, 63);
    }
    return v;
}

// What lane b of this lane's group holds (G >= 16, b a constant): lane b of
// every group is read into a scalar register and this group's is selected.
template <int G>
__device__ __forceinline__ uint32_t group_lane(uint32_t v, int b) {
    static_assert(G >= 16 && G <= 64, "group_lane: groups of 16 to 64 lanes");
    uint32_t r = (uint32_t)__builtin_amdgcn_readlane((int)v, b);
    if constexpr (G < 64) {
        const int grp = (int)__lane_id() / G;
#pragma unroll
        for (int g = 1; g < 64 / G; ++g) {
            const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)v, g * G + b);
            r = grp == g ? o : r;
        }
    }
    return r;
}

// A copy of v that the compiler treats as varying across lanes.  A value
// loaded through a uniform address is uniform, and the compiler moves it to
// scalar registers as soon as the load returns, which makes the wave wait for
// that load where it is issued; row indices pass through here after the draw
// so that the records loaded through them stay in vector registers and are
// waited for where they are used.
__device__ __forceinline__ uint32_t as_varying(uint32_t v) {
    uint32_t r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// A value that is the same in every active lane, moved to a scalar register
// (so that arithmetic on it runs on the scalar unit).
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Units per lane kept in registers: a row of up to G * UPL units is read
// once; longer rows are read twice (dot pass, then scatter pass).
template <int G> struct Upl { static constexpr int value = G >= 8 ? 1 : 8 / G; };

// ---------------------------------------------------------------- sweep

// One ticket of one worker (a group of G lanes): draw the row, fetch its
// record, gather-dot, step, atomic scatter.  XK: iterate dtype.  FP32 records
// with an FP64 iterate read b_i and 1/w_i in FP64 from the side array (the
// record header holds them in FP32).  With SAMPLED = false the row is
// `given_row` (the slice scheme).  tp (nullable): when tp->sample is set, the
// completion counter and the clock are read just before the gathers and
// just before the scatter.
template <int VK, int XK, int G, int UPL = Upl<G>::value, bool SAMPLED = true>
__device__ __forceinline__ void process_ticket(
    const Rows &rows, typename std::conditional<XK == ASYRK_F64, double, float>::type *x, int xsh,
    const double2 *side, int64_t j, uint32_t stream_id, uint32_t k0, uint32_t k1, int uniform,
    int update_one, typename std::conditional<XK == ASYRK_F64, double, float>::type gamma, int gl,
    TauProbe *tp, uint32_t given_row = 0) {
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

    if (tp && tp->sample) {
        tp->c0 = tau_read(tp->ctr);
        tp->t0 = wall_clock64();
    }

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
                    if (uu * U + e < nnz) acc = fma((X)un[q].v[e], load_agent(xat(x, un[q].c[e], xsh)), acc);
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
                        if (uu * U + e < nnz) acc = fma((X)un[q].v[e], load_agent(xat(x, un[q].c[e], xsh)), acc);
                }
            }
        }
    }
    acc = group_sum<G>(acc);

    // a4: step s = gamma * (a_i^T x - b_i) / ||a_i||^2
    X bi, inv_w;
    if constexpr (SIDE) {
        const double2 sd = gload<double2>(side + i);
        bi = sd.x;
        inv_w = sd.y;
    } else {
        bi = (X)h.b;
        inv_w = (X)h.inv_w;
    }
    const X r = acc - bi;
    if (tp && tp->sample) {
        tp->c1 = tau_read(tp->ctr);
        tp->t1 = wall_clock64();
    }

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
                        if (uu * U + e < nnz) atomic_add(xat(x, un[q].c[e], xsh), -s * (X)un[q].v[e]);
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
                            if (uu * U + e < nnz) atomic_add(xat(x, un[q].c[e], xsh), -s * (X)un[q].v[e]);
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
        atomic_add(xat(x, c, xsh), -s1 * (X)v);
    }
}

// The tickets j0, j0 + step, ... < j_end of one worker with the steps of
// process_ticket (sampled rows, all-coordinate update), software pipelined
// so that a ticket costs about one memory round trip instead of one per
// access.  For ticket t:
//
//   1. t's gathers are issued back to back (padded slots read x[0] and are
//      masked out by a select, so no branch splits them);
//   2. t+1's record is requested (its row locator arrived during t-1), then
//      t+2's locator;
//   3. t's gathers are consumed: the wait covers them only, not the loads of
//      step 2, which were issued later;
//   4. t's atomics are issued, with no load waited for between them;
//   5. t+1's alias decision needs its record header: that wait covers loads
//      issued before t's atomics only, so t+1's gathers leave while t's
//      atomics are still in flight.
//
// Row records are read-only during a sweep, so fetching them early moves no
// read of x.  A worker's gathers for t+1 follow its atomics for t in program
// order; the memory system keeps one wave's accesses to one address in order,
// so the worker still sees its own update (the one-worker pipelined run
// equals the sequential oracle to 1e-12).
//
// The row of a ticket comes from `pick(j, i)`, which returns the ticket's
// random words and sets its bucket row i: the Philox draw for sampled rows
// (SampledPick), or a row given outright with uniform = 1 (a slice walk).
//
// TRACE: on the sampled steps (see TauProbe) the completion counter is read
// as the gathers leave and again just before the scatter is issued.  Both
// reads sit in branches on the same wave-uniform step number, and their values
// are taken where the loop waits anyway: the first with the gathers, the
// second with the wait for the next ticket's record header (step 5), which
// covers every load issued before the atomics.  Nothing is carried across
// iterations unwaited (a loaded value live across the loop's back edge is
// copied there, and the copy waits for everything issued before it, the
// atomics included).
template <int VK, int XK, int G, int UPL, bool TRACE = false, class Pick>
__device__ __forceinline__ void run_rows_pipelined(
    const Rows rows, typename std::conditional<XK == ASYRK_F64, double, float>::type *x, int xsh,
    const double2 *side, int64_t j, int64_t j_end, int64_t step, int uniform,
    typename std::conditional<XK == ASYRK_F64, double, float>::type gamma, int gl, const Pick pick,
    uint64_t *tau_ctr = nullptr, int64_t wave = 0, TauAcc *tacc = nullptr) {
    using T = VT<VK>;
    using X = typename std::conditional<XK == ASYRK_F64, double, float>::type;
    using H = typename T::hdr_t;
    constexpr bool SIDE = (XK == ASYRK_F64) && (VK != ASYRK_F64);
    constexpr int U = T::U;
    if constexpr (G == 64) {
        // a worker is a whole wave: its tickets, and so its draws, are scalar
        j = wave_uniform(j);
        j_end = wave_uniform(j_end);
        step = wave_uniform(step);
    }
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
    // branch-free gathers of one chunk held in registers, issued ...
    auto gather_issue = [&](const Unit<VK> *cu, int base, int nnz, X (*xv)[U], X *(*xa)[U]) {
#pragma unroll
        for (int q = 0; q < UPL; ++q)
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const bool ok = (base + gl + q * G) * U + e < nnz;
                xa[q][e] = xat(x, ok ? cu[q].c[e] : 0, xsh);
                xv[q][e] = load_agent(xa[q][e]);
            }
    };
    // ... and consumed
    auto gather_dot = [&](const Unit<VK> *cu, int base, int nnz, X (*xv)[U], X acc) {
#pragma unroll
        for (int q = 0; q < UPL; ++q)
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const bool ok = (base + gl + q * G) * U + e < nnz;
                acc = ok ? fma((X)cu[q].v[e], xv[q][e], acc) : acc;
            }
        return acc;
    };
    // the scatter of a chunk whose gathers computed the addresses xa
    auto chunk_scatter = [&](const Unit<VK> *cu, X *(*xa)[U], int base, int nnz, X s) {
#pragma unroll
        for (int q = 0; q < UPL; ++q)
#pragma unroll
            for (int e = 0; e < U; ++e)
                if ((base + gl + q * G) * U + e < nnz) atomic_add(xa[q][e], -s * (X)cu[q].v[e]);
    };
    // the scatter of a chunk re-read from the record (long rows)
    auto chunk_scatter_reread = [&](const Unit<VK> *cu, int base, int nnz, X s) {
#pragma unroll
        for (int q = 0; q < UPL; ++q)
#pragma unroll
            for (int e = 0; e < U; ++e)
                if ((base + gl + q * G) * U + e < nnz) atomic_add(xat(x, cu[q].c[e], xsh), -s * (X)cu[q].v[e]);
    };
    // a row's locator is loaded in one ticket and used in the next, so the
    // loaded word is carried raw (a value used at once would be waited for at once)
    auto locator_load = [&](uint32_t r) -> RowLoc {
        return gload<RowLoc>(rows.loc != nullptr ? (const void *)(rows.loc + r) : (const void *)kZeroPad);
    };
    auto from_locator = [&](uint32_t r, const RowLoc &l, const uint8_t *&rec, int &nnz) {
        const bool ragged = rows.loc != nullptr;
        rec = ragged ? rows.rec + (int64_t)l.off16 * 16 : rows.rec + (int64_t)r * rows.stride;
        nnz = ragged ? (int)l.nnz : rows.fixed_nnz;
    };
    // the alias branch of the draw (needs the bucket row's header)
    auto resolve = [&](const U4 &u, uint32_t &i, const uint8_t *&rec, int &nnz, H &h, Unit<VK> *dst) {
        if (!uniform && !(u.c < h.thresh)) {
            i = (uint32_t)h.alias;
            locate_nb(rows, i, rec, nnz);
            h = load_hdr<VK>(rec);
            fetch_units(rec, (nnz + U - 1) / U, dst);
            return true;
        }
        return false;
    };

    // prologue: ticket j in full, ticket j + step's locator
    uint32_t i;
    U4 u = pick(j, i);
    i = as_varying(i);
    const uint8_t *rec;
    int nnz;
    locate_nb(rows, i, rec, nnz);
    H h = load_hdr<VK>(rec);
    Unit<VK> un[UPL];
    fetch_units(rec, (nnz + U - 1) / U, un);
    resolve(u, i, rec, nnz, h, un);
    X bi, inv_w;
    if constexpr (SIDE) {
        const double2 sd = gload<double2>(side + i);
        bi = sd.x;
        inv_w = sd.y;
    } else {
        bi = (X)h.b;
        inv_w = (X)h.inv_w;
    }
    // (tickets drawn past the end have valid rows and are simply not used)
    uint32_t i1;
    U4 u1 = pick(j + step, i1);
    i1 = as_varying(i1);
    RowLoc l1 = locator_load(i1);

    // staleness samples (TRACE)
    int64_t nstep = 0;
    uint32_t mine = 0;  // this worker's rows not yet added to the counter
    uint64_t c0v[kTauShards], c1v[kTauShards];

    for (;;) {
        const int64_t jn = j + step;
        const bool more = jn < j_end;
        const int nunits = (nnz + U - 1) / U;
        const bool samp = TRACE && (nstep % kTauPeriod == kTauFlush);
        uint64_t t0 = 0, t1 = 0;
        // 1. this ticket's gathers
        X xv[UPL][U];
        X *xa[UPL][U];
        gather_issue(un, 0, nnz, xv, xa);
        if constexpr (TRACE) {
            // (right behind the gathers: a branch before them would make the
            // wait for this ticket's units at their issue a wait for everything)
            if (samp) {
                tau_issue(tau_ctr, c0v);
                t0 = wall_clock64();
            }
        }
        // 2. the next ticket's record, then the locator of the one after
        const uint8_t *rec1;
        int nnz1;
        from_locator(i1, l1, rec1, nnz1);
        // (with side records only the sampling fields are read: loading the
        // unused b_i, 1/w_i lets the allocator reuse their registers while
        // the load is in flight, which forces a wait for everything)
        H h1;
        if constexpr (SIDE) {
            const gv2u ta = gload<gv2u>(rec1 + offsetof(H, thresh));
            h1.thresh = ta.x;
            h1.alias = (int32_t)ta.y;
        } else {
            h1 = load_hdr<VK>(rec1);
        }
        Unit<VK> un1[UPL];
        fetch_units(rec1, (nnz1 + U - 1) / U, un1);
        double2 sd1{0.0, 0.0};
        if constexpr (SIDE) sd1 = gload<double2>(side + i1);
        uint32_t i2;
        const U4 u2 = pick(jn + step, i2);
        i2 = as_varying(i2);
        const RowLoc l2 = locator_load(i2);
        // 3. gather-dot: the first chunk from registers (waiting for these
        // gathers only), then further chunks of long rows, re-read after it so
        // that neither a loop entry nor its exit joins the wait above
        X acc = gather_dot(un, 0, nnz, xv, (X)0);
        for (int base = G * UPL; base < nunits; base += G * UPL) {
            Unit<VK> t[UPL];
            fetch_chunk(rec, base, nunits, t);
            X tv[UPL][U];
            X *ta[UPL][U];
            gather_issue(t, base, nnz, tv, ta);
            acc = gather_dot(t, base, nnz, tv, acc);
        }
        acc = group_sum<G>(acc);
        if constexpr (TRACE) {
            if (samp) {
                tau_issue(tau_ctr, c1v);
                t1 = wall_clock64();
            }
        }
        const X s = gamma * (acc - bi) * inv_w;
        // 4. lock-free scatter
        chunk_scatter(un, xa, 0, nnz, s);
        for (int base = G * UPL; base < nunits; base += G * UPL) {
            Unit<VK> t[UPL];
            fetch_chunk(rec, base, nunits, t);
            chunk_scatter_reread(t, base, nnz, s);
        }
        if constexpr (TRACE) {
            ++mine;
            if (nstep % kTauFlush == kTauFlush - 1) tau_flush_wave(tau_ctr, wave, gl, mine);
            ++nstep;
        }
        if (!more) {
            if constexpr (TRACE) {
                if (samp) tau_accumulate(*tacc, tau_sum(c0v), tau_sum(c1v), t0, t1);
                tau_flush_leader(tau_ctr, wave, gl, mine);
            }
            break;
        }
        // 5. rotate: the next ticket becomes current
        if (resolve(u1, i1, rec1, nnz1, h1, un1)) {
            if constexpr (SIDE) sd1 = gload<double2>(side + i1);
        }
        if constexpr (TRACE) {
            // the header wait above covered the counter loads issued before the atomics
            if (samp) tau_accumulate(*tacc, tau_sum(c0v), tau_sum(c1v), t0, t1);
        }
        if constexpr (SIDE) {
            bi = sd1.x;
            inv_w = sd1.y;
        } else {
            bi = (X)h1.b;
            inv_w = (X)h1.inv_w;
        }
        j = jn;
        i = i1;
        rec = rec1;
        nnz = nnz1;
#pragma unroll
        for (int q = 0; q < UPL; ++q) un[q] = un1[q];
        u1 = u2;
        i1 = i2;
        l1 = l2;
    }
}

// s_waitcnt immediate (gfx9 encoding) for vmcnt(0) alone: expcnt(7) and
// lgkmcnt(15) are their maxima, i.e. no wait on those counters.
constexpr int kWaitVmcnt0 = 0x0F70;

// Tickets per batch of the batched worker loop: B records held in registers,
// so fewer for wider rows per lane (units per lane UPL).
template <int UPL> struct BatchOf { static constexpr int value = UPL == 1 ? 8 : (UPL == 2 ? 4 : 2); };

// The same tickets as run_rows_pipelined (all-coordinate update, rows from
// `pick`), with the row records fetched in batches.  A wave's vector loads
// complete in order, so a wait for a ticket's gathers is also a wait for
// every record requested before them: a record requested one ticket ahead
// puts an HBM round trip on every ticket, whatever else overlaps it.  Here
// the only loads between batch boundaries are the tickets' own gathers (and
// the extra chunks of long rows).  At a boundary the wave requests the
// records of the next B tickets, whose locators arrived at the previous
// boundary, together with the draws' locators of the batch after, waits for
// them once, takes the alias decisions (a taken alias re-reads its row and
// waits for it), and then runs the B tickets back to back: gathers, wait,
// dot, atomics.  One record round trip per B tickets instead of per ticket.
// Reads of x happen exactly where the other loops make them (after the
// worker's previous atomics, in program order), so a lone worker still
// equals the sequential oracle.  TRACE as in run_rows_pipelined.
template <int VK, int XK, int G, int UPL, bool TRACE, class Pick>
__device__ __forceinline__ void run_rows_batched(
    const Rows rows, typename std::conditional<XK == ASYRK_F64, double, float>::type *x, int xsh,
    const double2 *side, int64_t j, int64_t j_end, int64_t step, int uniform,
    typename std::conditional<XK == ASYRK_F64, double, float>::type gamma, int gl, const Pick pick,
    uint64_t *tau_ctr = nullptr, int64_t wave = 0, TauAcc *tacc = nullptr) {
    using T = VT<VK>;
    using X = typename std::conditional<XK == ASYRK_F64, double, float>::type;
    using H = typename T::hdr_t;
    constexpr bool SIDE = (XK == ASYRK_F64) && (VK != ASYRK_F64);
    constexpr int U = T::U;
    constexpr int B = BatchOf<UPL>::value;
    if constexpr (G == 64) {
        j = wave_uniform(j);
        j_end = wave_uniform(j_end);
        step = wave_uniform(step);
    }
    if (j >= j_end) return;

    static_assert(T::UB <= (int)sizeof(kZeroPad), "zero pad smaller than a unit");
    auto fetch_chunk = [&](const uint8_t *rec, int base, int nunits, Unit<VK> *dst) {
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int uu = base + gl + q * G;
            dst[q].load(uu < nunits ? rec + T::HB + (int64_t)uu * T::UB : kZeroPad);
        }
    };
    auto gather_issue = [&](const Unit<VK> *cu, int base, int nnz, X (*xv)[U], X *(*xa)[U]) {
#pragma unroll
        for (int q = 0; q < UPL; ++q)
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const bool ok = (base + gl + q * G) * U + e < nnz;
                xa[q][e] = xat(x, ok ? cu[q].c[e] : 0, xsh);
                xv[q][e] = load_agent(xa[q][e]);
            }
    };
    auto gather_dot = [&](const Unit<VK> *cu, int base, int nnz, X (*xv)[U], X acc) {
#pragma unroll
        for (int q = 0; q < UPL; ++q)
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const bool ok = (base + gl + q * G) * U + e < nnz;
                acc = ok ? fma((X)cu[q].v[e], xv[q][e], acc) : acc;
            }
        return acc;
    };
    // the scatter of a chunk whose gathers computed the addresses xa
    auto chunk_scatter = [&](const Unit<VK> *cu, X *(*xa)[U], int base, int nnz, X s) {
#pragma unroll
        for (int q = 0; q < UPL; ++q)
#pragma unroll
            for (int e = 0; e < U; ++e)
                if ((base + gl + q * G) * U + e < nnz) atomic_add(xa[q][e], -s * (X)cu[q].v[e]);
    };
    // the scatter of a chunk re-read from the record (long rows)
    auto chunk_scatter_reread = [&](const Unit<VK> *cu, int base, int nnz, X s) {
#pragma unroll
        for (int q = 0; q < UPL; ++q)
#pragma unroll
            for (int e = 0; e < U; ++e)
                if ((base + gl + q * G) * U + e < nnz) atomic_add(xat(x, cu[q].c[e], xsh), -s * (X)cu[q].v[e]);
    };
    auto locator_load = [&](uint32_t r) -> RowLoc {
        return gload<RowLoc>(rows.loc != nullptr ? (const void *)(rows.loc + r) : (const void *)kZeroPad);
    };
    auto from_locator = [&](uint32_t r, const RowLoc &l, const uint8_t *&rec, int &nnz) {
        const bool ragged = rows.loc != nullptr;
        rec = ragged ? rows.rec + (int64_t)l.off16 * 16 : rows.rec + (int64_t)r * rows.stride;
        nnz = ragged ? (int)l.nnz : rows.fixed_nnz;
    };

    // the batch in registers: slot b holds ticket jb + b * step
    uint32_t si[B], suc[B];
    const uint8_t *srec[B];
    int snnz[B];
    H sh[B];
    Unit<VK> sun[B][UPL];
    double2 ssd[B];
    X sbi[B], sinv[B];
    // the next batch's draws and locators
    uint32_t ni[B], nuc[B];
    RowLoc nl[B];

    // the draws and locators of the batch that starts at ticket jn.  With
    // G >= 16 lane b of a group draws ticket jn + b * step (one pass of the
    // generator for the whole batch) and every lane reads its group's B draws
    // back; narrower groups draw ticket by ticket.
    auto draw_batch = [&](int64_t jn) {
        if constexpr (G >= 16) {
            uint32_t il;
            const U4 ul = pick(jn + (int64_t)(gl % B) * step, il);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                ni[b] = as_varying(group_lane<G>(il, b));
                nuc[b] = group_lane<G>(ul.c, b);
                nl[b] = locator_load(ni[b]);
            }
        } else {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                nuc[b] = pick(jn + (int64_t)b * step, ni[b]).c;
                nl[b] = locator_load(ni[b]);
            }
        }
    };
    // the records of the batch whose locators arrived, then the draws and
    // locators of the batch after it (first ticket jn), all requested together
    auto request_batch = [&](int64_t jn) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            si[b] = ni[b];
            suc[b] = nuc[b];
            from_locator(si[b], nl[b], srec[b], snnz[b]);
            if constexpr (SIDE) {
                const gv2u ta = gload<gv2u>(srec[b] + offsetof(H, thresh));
                sh[b].thresh = ta.x;
                sh[b].alias = (int32_t)ta.y;
            } else {
                sh[b] = load_hdr<VK>(srec[b]);
            }
            fetch_chunk(srec[b], 0, (snnz[b] + U - 1) / U, sun[b]);
            if constexpr (SIDE) ssd[b] = gload<double2>(side + si[b]);
        }
        draw_batch(jn);
    };
    // the alias decisions of the batch (its loads have arrived), then b_i, 1/w_i
    auto resolve_batch = [&]() {
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (!uniform && !(suc[b] < sh[b].thresh)) {
                si[b] = (uint32_t)sh[b].alias;
                locate_nb(rows, si[b], srec[b], snnz[b]);
                sh[b] = load_hdr<VK>(srec[b]);
                fetch_chunk(srec[b], 0, (snnz[b] + U - 1) / U, sun[b]);
                if constexpr (SIDE) ssd[b] = gload<double2>(side + si[b]);
                __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            }
            if constexpr (SIDE) {
                sbi[b] = ssd[b].x;
                sinv[b] = ssd[b].y;
            } else {
                sbi[b] = (X)sh[b].b;
                sinv[b] = (X)sh[b].inv_w;
            }
        }
    };

    // prologue: the first batch's draws and locators
    draw_batch(j);
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);

    int64_t nstep = 0;
    uint32_t mine = 0;
    uint64_t c0v[kTauShards], c1v[kTauShards];
    for (;;) {
        request_batch(j + (int64_t)B * step);
        resolve_batch();
        bool done = false;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (!done) {
                const int nnz = snnz[b];
                const int nunits = (nnz + U - 1) / U;
                const bool samp = TRACE && (nstep % kTauPeriod == kTauFlush);
                uint64_t t0 = 0, t1 = 0;
                X xv[UPL][U];
                X *xa[UPL][U];
                gather_issue(sun[b], 0, nnz, xv, xa);
                if constexpr (TRACE) {
                    if (samp) {
                        tau_issue(tau_ctr, c0v);
                        t0 = wall_clock64();
                    }
                }
                X acc = gather_dot(sun[b], 0, nnz, xv, (X)0);
                for (int base = G * UPL; base < nunits; base += G * UPL) {
                    Unit<VK> tu[UPL];
                    fetch_chunk(srec[b], base, nunits, tu);
                    X tv[UPL][U];
                    X *ta[UPL][U];
                    gather_issue(tu, base, nnz, tv, ta);
                    acc = gather_dot(tu, base, nnz, tv, acc);
                }
                acc = group_sum<G>(acc);
                if constexpr (TRACE) {
                    if (samp) {
                        tau_issue(tau_ctr, c1v);
                        t1 = wall_clock64();
                    }
                }
                const X s = gamma * (acc - sbi[b]) * sinv[b];
                chunk_scatter(sun[b], xa, 0, nnz, s);
                for (int base = G * UPL; base < nunits; base += G * UPL) {
                    Unit<VK> tu[UPL];
                    fetch_chunk(srec[b], base, nunits, tu);
                    chunk_scatter_reread(tu, base, nnz, s);
                }
                if constexpr (TRACE) {
                    ++mine;
                    if (nstep % kTauFlush == kTauFlush - 1) tau_flush_wave(tau_ctr, wave, gl, mine);
                    ++nstep;
                    if (samp) tau_accumulate(*tacc, tau_sum(c0v), tau_sum(c1v), t0, t1);
                }
                j += step;
                done = j >= j_end;
            }
        }
        if (done) break;
    }
    if constexpr (TRACE) tau_flush_leader(tau_ctr, wave, gl, mine);
}

// Sampled rows: ticket j's Philox draw and its bucket.
struct SampledPick {
    uint32_t m, stream_id, k0, k1;
    __device__ __forceinline__ U4 operator()(int64_t j, uint32_t &i) const {
        const U4 u = draw(j, stream_id, k0, k1);
        i = bucket_of(u.a, u.b, m);
        return u;
    }
};

template <int VK, int XK, int G, int UPL = Upl<G>::value, bool TRACE = false>
__device__ __forceinline__ void run_tickets_pipelined(
    const Rows rows, typename std::conditional<XK == ASYRK_F64, double, float>::type *x, int xsh,
    const double2 *side, int64_t j, int64_t j_end, int64_t step, uint32_t stream_id, uint32_t k0,
    uint32_t k1, int uniform, typename std::conditional<XK == ASYRK_F64, double, float>::type gamma,
    int gl, uint64_t *tau_ctr = nullptr, int64_t wave = 0, TauAcc *tacc = nullptr) {
    run_rows_pipelined<VK, XK, G, UPL, TRACE>(rows, x, xsh, side, j, j_end, step, uniform, gamma, gl,
                                              SampledPick{(uint32_t)rows.m, stream_id, k0, k1}, tau_ctr,
                                              wave, tacc);
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

// The slice walk of one worker as tickets 0, 1, ...: ticket t is position
// k = t mod L of sweep sw0 + t / L in the worker's keyed permutation of its
// rows [start, start + L) (L >= 1).
struct SlicePick {
    int64_t start, sw0;
    uint32_t L, worker, k0, k1;
    __device__ __forceinline__ U4 operator()(int64_t t, uint32_t &i) const {
        uint64_t sw, k;
        if ((uint64_t)t >> 32 == 0) {
            sw = (uint32_t)t / L;
            k = (uint32_t)t - (uint32_t)sw * L;
        } else {
            sw = (uint64_t)t / L;
            k = (uint64_t)t - sw * L;
        }
        sw += (uint64_t)sw0;
        const U4 u = philox4x32_10((uint32_t)(sw & 0xffffffffu), (uint32_t)(sw >> 32), worker, 0x5C4E3D2Bu, k0, k1);
        i = (uint32_t)(start + slice_perm((uint32_t)k, L, u));
        return U4{0u, 0u, 0u, 0u};
    }
};

// ---------------------------------------------------------------- split worker
//
// A wave-wide worker (G = 64) split over two waves of one workgroup: the
// fetch wave draws the rows of a batch of tickets, loads their locators and
// records, takes the alias decisions and leaves each ticket's units and
// scalars in LDS; the compute wave runs the tickets from LDS: gathers, dot,
// sum, step, atomics.  The two alternate between two LDS buffers, one
// barrier per batch: while the compute wave runs batch k, the fetch wave
// fills the other buffer with batch k + 1.  The compute wave then issues no
// record or locator loads of its own (rows longer than 64 units aside), so
// its waits on the vector memory counter are for its gathers and its earlier
// atomics only; LDS reads are counted apart.  Its reads of x happen where the
// other loops make them (after the worker's previous atomics, in program
// order), so a lone worker equals the sequential oracle.  Both waves run the
// same number of batches, from values uniform over the workgroup, and pass
// the same barriers; neither leaves the loop early.

template <int VK> struct SplitBatch { static constexpr int value = VK == ASYRK_BF16 ? 4 : 8; };

// One ticket's scalars in LDS (the units sit in their own array).
template <int XK> struct SplitMeta {
    using X = typename std::conditional<XK == ASYRK_F64, double, float>::type;
    const uint8_t *rec;
    int nnz;
    X bi, inv_w;
};

// Barrier of the two waves of a split worker; the fences order LDS only, so
// the compute wave does not wait for its atomics here.
__device__ __forceinline__ void split_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// role 0: compute wave, 1: fetch wave; lane = the lane in the wave.  j, j_end
// and step must be the same in both waves.  lu / lm: the workgroup's two
// batch buffers.
template <int VK, int XK, bool TRACE, class Pick>
__device__ __forceinline__ void run_rows_split(
    const Rows rows, typename std::conditional<XK == ASYRK_F64, double, float>::type *x, int xsh,
    const double2 *side, int64_t j, int64_t j_end, int64_t step, int uniform,
    typename std::conditional<XK == ASYRK_F64, double, float>::type gamma, int role, int lane, const Pick pick,
    Unit<VK> (*lu)[SplitBatch<VK>::value][64], SplitMeta<XK> (*lm)[SplitBatch<VK>::value],
    uint64_t *tau_ctr = nullptr, int64_t wave = 0, TauAcc *tacc = nullptr) {
    using T = VT<VK>;
    using X = typename std::conditional<XK == ASYRK_F64, double, float>::type;
    using H = typename T::hdr_t;
    constexpr bool SIDE = (XK == ASYRK_F64) && (VK != ASYRK_F64);
    constexpr int G = 64;
    constexpr int U = T::U;
    constexpr int B = SplitBatch<VK>::value;
    j = wave_uniform(j);
    j_end = wave_uniform(j_end);
    step = wave_uniform(step);
    const int64_t span = (int64_t)B * step;
    const int64_t nb = j < j_end ? (j_end - j + span - 1) / span : 0;
    if (nb == 0) return;  // both waves alike, before any barrier

    static_assert(T::UB <= (int)sizeof(kZeroPad), "zero pad smaller than a unit");
    auto unit_at = [&](const uint8_t *rec, int uu, int nunits) -> const uint8_t * {
        return uu < nunits ? rec + T::HB + (int64_t)uu * T::UB : kZeroPad;
    };

    if (role == 1) {
        // ---- fetch wave: batch jb into buffer buf
        auto fetch = [&](int64_t jb, int buf) {
            uint32_t il;
            const U4 ul = pick(jb + (int64_t)(lane % B) * step, il);
            uint32_t ri[B], ru[B];
            RowLoc rl[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                ri[b] = as_varying(group_lane<G>(il, b));
                ru[b] = group_lane<G>(ul.c, b);
                rl[b] = gload<RowLoc>(rows.loc != nullptr ? (const void *)(rows.loc + ri[b]) : (const void *)kZeroPad);
            }
            const uint8_t *rec[B];
            int nnz[B];
            H h[B];
            Unit<VK> un[B];
            double2 sd[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const bool ragged = rows.loc != nullptr;
                rec[b] = ragged ? rows.rec + (int64_t)rl[b].off16 * 16 : rows.rec + (int64_t)ri[b] * rows.stride;
                nnz[b] = ragged ? (int)rl[b].nnz : rows.fixed_nnz;
                h[b] = load_hdr<VK>(rec[b]);
                un[b].load(unit_at(rec[b], lane, (nnz[b] + U - 1) / U));
                if constexpr (SIDE) sd[b] = gload<double2>(side + ri[b]);
            }
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (!uniform && !(ru[b] < h[b].thresh)) {
                    ri[b] = (uint32_t)h[b].alias;
                    locate_nb(rows, ri[b], rec[b], nnz[b]);
                    h[b] = load_hdr<VK>(rec[b]);
                    un[b].load(unit_at(rec[b], lane, (nnz[b] + U - 1) / U));
                    if constexpr (SIDE) sd[b] = gload<double2>(side + ri[b]);
                }
                lu[buf][b][lane] = un[b];
                if (lane == 0) {
                    SplitMeta<XK> mt;
                    mt.rec = rec[b];
                    mt.nnz = nnz[b];
                    if constexpr (SIDE) {
                        mt.bi = sd[b].x;
                        mt.inv_w = sd[b].y;
                    } else {
                        mt.bi = (X)h[b].b;
                        mt.inv_w = (X)h[b].inv_w;
                    }
                    lm[buf][b] = mt;
                }
            }
        };
        fetch(j, 0);
        split_barrier();
        for (int64_t k = 0; k < nb; ++k) {
            if (k + 1 < nb) fetch(j + (k + 1) * span, (int)((k + 1) & 1));
            split_barrier();
        }
        return;
    }

    // ---- compute wave
    auto gather_issue = [&](const Unit<VK> &cu, int base, int nnz, X *xv, X **xa) {
#pragma unroll
        for (int e = 0; e < U; ++e) {
            const bool ok = (base + lane) * U + e < nnz;
            xa[e] = xat(x, ok ? cu.c[e] : 0, xsh);
            xv[e] = load_agent(xa[e]);
        }
    };
    auto gather_dot = [&](const Unit<VK> &cu, int base, int nnz, const X *xv, X acc) {
#pragma unroll
        for (int e = 0; e < U; ++e) {
            const bool ok = (base + lane) * U + e < nnz;
            acc = ok ? fma((X)cu.v[e], xv[e], acc) : acc;
        }
        return acc;
    };
    auto scatter = [&](const Unit<VK> &cu, X *const *xa, int base, int nnz, X s) {
#pragma unroll
        for (int e = 0; e < U; ++e)
            if ((base + lane) * U + e < nnz) atomic_add(xa[e], -s * (X)cu.v[e]);
    };
    auto scatter_reread = [&](const Unit<VK> &cu, int base, int nnz, X s) {
#pragma unroll
        for (int e = 0; e < U; ++e)
            if ((base + lane) * U + e < nnz) atomic_add(xat(x, cu.c[e], xsh), -s * (X)cu.v[e]);
    };

    split_barrier();  // batch 0 is in buffer 0
    int64_t nstep = 0;
    uint32_t mine = 0;
    uint64_t c0v[kTauShards], c1v[kTauShards];
    for (int64_t k = 0; k < nb; ++k) {
        const int buf = (int)(k & 1);
        const int64_t jb = j + k * span;
        Unit<VK> cu = lu[buf][0][lane];
        SplitMeta<XK> mt = lm[buf][0];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (jb + (int64_t)b * step < j_end) {
                const int nnz = mt.nnz;
                const int nunits = (nnz + U - 1) / U;
                const bool samp = TRACE && (nstep % kTauPeriod == kTauFlush);
                uint64_t t0 = 0, t1 = 0;
                X xv[U];
                X *xa[U];
                gather_issue(cu, 0, nnz, xv, xa);
                if constexpr (TRACE) {
                    if (samp) {
                        tau_issue(tau_ctr, c0v);
                        t0 = wall_clock64();
                    }
                }
                // the next ticket's unit and scalars, read from LDS while
                // these gathers are in flight (LDS reads wait on their own
                // counter)
                Unit<VK> ncu = cu;
                SplitMeta<XK> nmt = mt;
                if (b + 1 < B) {
                    ncu = lu[buf][b + 1][lane];
                    nmt = lm[buf][b + 1];
                }
                X acc = gather_dot(cu, 0, nnz, xv, (X)0);
                for (int base = G; base < nunits; base += G) {
                    Unit<VK> tu;
                    tu.load(unit_at(mt.rec, base + lane, nunits));
                    X tv[U];
                    X *ta[U];
                    gather_issue(tu, base, nnz, tv, ta);
                    acc = gather_dot(tu, base, nnz, tv, acc);
                }
                acc = group_sum<G>(acc);
                if constexpr (TRACE) {
                    if (samp) {
                        tau_issue(tau_ctr, c1v);
                        t1 = wall_clock64();
                    }
                }
                const X s = gamma * (acc - mt.bi) * mt.inv_w;
                scatter(cu, xa, 0, nnz, s);
                for (int base = G; base < nunits; base += G) {
                    Unit<VK> tu;
                    tu.load(unit_at(mt.rec, base + lane, nunits));
                    scatter_reread(tu, base, nnz, s);
                }
                if constexpr (TRACE) {
                    ++mine;
                    if (nstep % kTauFlush == kTauFlush - 1) tau_flush_wave(tau_ctr, wave, lane, mine);
                    ++nstep;
                    if (samp) tau_accumulate(*tacc, tau_sum(c0v), tau_sum(c1v), t0, t1);
                }
                cu = ncu;
                mt = nmt;
            }
        }
        split_barrier();  // buffer buf is free again; the next batch is in the other one
    }
    if constexpr (TRACE) tau_flush_leader(tau_ctr, wave, lane, mine);
}

}  // namespace asyrk
