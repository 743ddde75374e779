// Internal definitions shared by the host runtime and the gfx950 kernels of
// the asynchronous randomized Kaczmarz library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/asyrk.h"
#include "layout.h"

namespace asyrk {

// Geometry of the packed rows, passed by value to every kernel.
struct Rows {
    const uint8_t *rec;    // record base
    const RowLoc *loc;     // nullptr when every row has fixed_nnz entries
    int64_t stride;        // bytes between records when loc == nullptr
    int32_t fixed_nnz;     // common length when loc == nullptr
    int32_t m;
};

// Bytes per element of a sweep iterate over n columns.  Gathers and atomics
// on columns that share a cache line queue behind each other in the memory
// system, so the iterate is spread out when that costs little memory: a line
// of its own per column up to 2^20 columns (256 MB), 64 bytes up to 2^23,
// dense beyond.
inline int64_t iterate_stride(int64_t n) {
    if (n <= ((int64_t)1 << 20)) return 256;
    if (n <= ((int64_t)1 << 23)) return 64;
    return 8;
}

// log2(stride_bytes / elem_bytes) for power-of-two sizes
inline int stride_shift(int64_t stride_bytes, int elem_bytes) {
    int sh = 0;
    while (((int64_t)elem_bytes << sh) < stride_bytes) ++sh;
    return sh;
}

// Arguments of the sweep kernel.
struct SweepArgs {
    Rows rows;
    void *x;               // iterate: element c at x[c << xshift] (float or double)
    int32_t xshift;        // log2 of the iterate's element stride
    const double2 *side;   // FP64 iterate over FP32/BF16 records: {b_i, 1/w_i} per row
    int64_t t_begin;       // first ticket
    int64_t t_end;         // one past the last ticket
    int64_t R;             // row workers
    uint32_t key0, key1;   // Philox key (seed)
    uint32_t stream_id;
    int32_t uniform;       // 1: P(i) = 1/m
    int32_t update_one;    // 1: Algorithm 1 single-coordinate step
    int32_t replay;        // 1: wait for the scatter before the next read
    double gamma;
    uint64_t *trace;       // nullable: staleness samples, kTraceWords words per wave (device.h)
    uint64_t *tau_ctr;     // the completion counter's shards when trace is set
    int32_t slices;        // 1: without-replacement slice scheme (t_begin, t_end are sweep multiples)
    int32_t pipe;          // worker loop (asynchronous, all-coordinate): 1 software-pipelined, 2 batched records
};

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 64-bit product is one multiply-add instruction (both halves)
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo_a = (uint32_t)pa, hi_a = (uint32_t)(pa >> 32);
        const uint32_t lo_b = (uint32_t)pb, hi_b = (uint32_t)(pb >> 32);
        const uint32_t n0 = hi_b ^ c1 ^ k0;
        const uint32_t n2 = hi_a ^ c3 ^ k1;
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// floor((hi * 2^32 + lo) * m / 2^64) for m < 2^31, exactly.
__device__ __forceinline__ uint32_t bucket_of(uint32_t lo, uint32_t hi, uint32_t m) {
    const uint64_t t = (uint64_t)lo * m;
    const uint64_t s = (uint64_t)hi * m + (t >> 32);
    return (uint32_t)(s >> 32);
}

// Draw for ticket j: u = Philox(counter (j lo, j hi, stream, 0), key (k0, k1)).
__device__ __forceinline__ U4 draw(int64_t j, uint32_t stream_id, uint32_t k0, uint32_t k1) {
    return philox4x32_10((uint32_t)((uint64_t)j & 0xffffffffu), (uint32_t)((uint64_t)j >> 32),
                         stream_id, 0u, k0, k1);
}

// ---------------------------------------------------------------------------
// Host-side launchers (kernels.hip).  All return hipError_t of the launch.
// ---------------------------------------------------------------------------
hipError_t launch_sweep(int vk, int xk, int G, const SweepArgs &a, hipStream_t st);
hipError_t launch_sweep_slices(int vk, int xk, int G, const SweepArgs &a, hipStream_t st);
hipError_t launch_build_side(int vk, const Rows &rows, const double *b64, double2 *side, hipStream_t st);
// xsh: log2 of the element stride of x (0 = dense; the sweep iterate has its own)
hipError_t launch_residual(int vk, const Rows &rows, const double *b64, const void *x, int x_is_f32, int xsh,
                           double *r_out, int write_rec_b, double *partials, int nblocks,
                           hipStream_t st, int rhs_from_rec = 0);
hipError_t launch_sumsq_diff(const void *x, int x_is_f32, int xsh, const double *xr, int64_t n,
                             double *partials, int nblocks, hipStream_t st);
hipError_t launch_finish_sum(const double *partials, int nparts, double *out, hipStream_t st);
hipError_t launch_cast_to_iter(const double *x64, void *xit, int xit_is_f32, int xsh, int64_t n, hipStream_t st);
hipError_t launch_iter_to_f64(const void *xit, int xit_is_f32, int xsh, double *x64, int64_t n, int accumulate,
                              hipStream_t st);
hipError_t launch_zero(void *p, int64_t bytes, hipStream_t st);
hipError_t launch_set_rec_b(int vk, const Rows &rows, const double *b64, hipStream_t st);
hipError_t launch_scatter_rows(int vk, const Rows &rows, const double *y, double *z, hipStream_t st);
hipError_t launch_scale(double *v, int64_t n, const double *norm2, hipStream_t st);
hipError_t launch_divide(const double *z, double d, double *out, int64_t n, hipStream_t st);  // out = z / d
hipError_t launch_random_fill(double *v, int64_t n, uint32_t k0, uint32_t k1, hipStream_t st);
hipError_t launch_sample_rows(int vk, const Rows &rows, int64_t ticket0, int64_t count, uint32_t k0, uint32_t k1,
                              uint32_t stream_id, int uniform, int32_t *rows_out, int32_t *coords_out,
                              hipStream_t st);
hipError_t probe_copy(int64_t bytes, int iters, double *gbps);
hipError_t probe_scatter(int64_t n, int64_t count, int dtype, int kind, int iters, double *per_s);

constexpr int kResidualBlocks = 2048;   // fixed grid: deterministic partial sums

}  // namespace asyrk
