// Device-side setup for systems handed over in device memory: validation,
// row weights and column statistics (the row sampling of Section 1 needs
// w_i = ||a_i||^2 for every row, Corollary 1's bound the largest column norm),
// then the row records, written from the caller's CSR arrays without a round
// trip through host memory.  One thread per row in both passes.
#include "setup_dev.h"

namespace asyrk {

namespace {

template <int VK> struct StoredVal;
template <> struct StoredVal<ASYRK_F64> {
    using type = double;
    __device__ static double promote(double v) { return v; }
};
template <> struct StoredVal<ASYRK_F32> {
    using type = float;
    __device__ static double promote(float v) { return (double)v; }
};
template <> struct StoredVal<ASYRK_BF16> {
    using type = uint16_t;
    __device__ static double promote(uint16_t v) { return (double)__uint_as_float((uint32_t)v << 16); }
};

__host__ __device__ constexpr int64_t grid_for(int64_t count) { return (count + 255) / 256; }

template <int VK>
__global__ __launch_bounds__(256) void scan_rows_kernel(int64_t m, int32_t n, const int64_t *row_ptr,
                                                         const int32_t *col,
                                                         const typename StoredVal<VK>::type *vals,
                                                         const double *b, double *w, uint32_t *col_cnt,
                                                         double *col_sq, uint32_t *flags) {
    // the host's left-to-right sum: every product and sum rounded on its own
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    uint32_t bad = __builtin_isfinite(b[i]) ? 0u : kBadRhs;
    const int64_t beg = row_ptr[i], end = row_ptr[i + 1];
    double s = 0.0;
    int32_t prev = -1;
    for (int64_t k = beg; k < end; ++k) {
        const int32_t c = col[k];
        if (c <= prev || c >= n) {
            bad |= kBadEntry;
            break;
        }
        prev = c;
        const double v = StoredVal<VK>::promote(vals[k]);
        if (!__builtin_isfinite(v)) {
            bad |= kBadEntry;
            break;
        }
        const double v2 = v * v;
        s = s + v2;
        atomicAdd(col_cnt + c, 1u);
        unsafeAtomicAdd(col_sq + c, v2);
    }
    w[i] = s;
    if (bad) atomicOr(flags, bad);
}

__global__ __launch_bounds__(256) void col_max_kernel(const uint32_t *col_cnt, const double *col_sq, int64_t n,
                                                       unsigned long long *out) {
    __shared__ unsigned long long red[2][4];
    unsigned long long mc = 0, ms = 0;  // non-negative doubles order as their bit patterns
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        mc = max(mc, (unsigned long long)col_cnt[j]);
        ms = max(ms, (unsigned long long)__double_as_longlong(col_sq[j]));
    }
    for (int d = 32; d >= 1; d >>= 1) {
        mc = max(mc, (unsigned long long)__shfl_xor((long long)mc, d));
        ms = max(ms, (unsigned long long)__shfl_xor((long long)ms, d));
    }
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) {
        red[0][wave] = mc;
        red[1][wave] = ms;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 4; ++q) {
            mc = max(mc, red[0][q]);
            ms = max(ms, red[1][q]);
        }
        atomicMax(out, mc);
        atomicMax(out + 1, ms);
    }
}

template <int VK>
__global__ __launch_bounds__(256) void write_records_kernel(int64_t m, const int64_t *row_ptr, const int32_t *col,
                                                             const typename StoredVal<VK>::type *vals,
                                                             const double *b, const RowAux *aux, int64_t stride,
                                                             const RowLoc *loc, uint8_t *rec) {
    using T = VT<VK>;
    using val_t = typename StoredVal<VK>::type;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    uint8_t *r = rec + (loc ? (int64_t)loc[i].off16 * 16 : i * stride);
    const RowAux a = aux[i];
    if constexpr (VK == ASYRK_F64) {
        *reinterpret_cast<HdrF64 *>(r) = HdrF64{b[i], a.inv_w, a.thresh, a.alias, 0};
    } else {
        *reinterpret_cast<HdrF32 *>(r) = HdrF32{(float)b[i], (float)a.inv_w, a.thresh, a.alias};
    }
    const int64_t beg = row_ptr[i], nnz = row_ptr[i + 1] - beg;
    uint8_t *u = r + T::HB;
    for (int64_t k = 0; k < nnz; k += T::U, u += T::UB) {
        int32_t *uc = reinterpret_cast<int32_t *>(u);
        val_t *uv = reinterpret_cast<val_t *>(u + T::COLB);
#pragma unroll
        for (int e = 0; e < T::U; ++e) {
            const bool in = k + e < nnz;
            uc[e] = in ? col[beg + k + e] : 0;
            uv[e] = in ? vals[beg + k + e] : (val_t)0;
        }
    }
    if (!loc)
        for (uint8_t *p = u; p < r + stride; p += 16) *reinterpret_cast<uint4 *>(p) = uint4{0u, 0u, 0u, 0u};
}

__global__ __launch_bounds__(256) void check_finite_kernel(const double *v, int64_t n, uint32_t *flags) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad |= !__builtin_isfinite(v[i]);
    if (bad) atomicOr(flags, kBadRhs);
}

}  // namespace

hipError_t launch_check_finite_dev(const double *v, int64_t n, uint32_t *flags, hipStream_t st) {
    const int64_t blocks = grid_for(n) < 1024 ? grid_for(n) : 1024;
    hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, st, v, n, flags);
    return hipGetLastError();
}

hipError_t launch_scan_rows_dev(int vk, int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
                                const void *vals, const double *b, double *w, uint32_t *col_cnt, double *col_sq,
                                uint32_t *flags, hipStream_t st) {
    const dim3 grid((unsigned)grid_for(m)), block(256);
    switch (vk) {
        case ASYRK_F64:
            hipLaunchKernelGGL(scan_rows_kernel<ASYRK_F64>, grid, block, 0, st, m, (int32_t)n, row_ptr, col,
                               static_cast<const double *>(vals), b, w, col_cnt, col_sq, flags);
            break;
        case ASYRK_F32:
            hipLaunchKernelGGL(scan_rows_kernel<ASYRK_F32>, grid, block, 0, st, m, (int32_t)n, row_ptr, col,
                               static_cast<const float *>(vals), b, w, col_cnt, col_sq, flags);
            break;
        case ASYRK_BF16:
            hipLaunchKernelGGL(scan_rows_kernel<ASYRK_BF16>, grid, block, 0, st, m, (int32_t)n, row_ptr, col,
                               static_cast<const uint16_t *>(vals), b, w, col_cnt, col_sq, flags);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_col_max_dev(const uint32_t *col_cnt, const double *col_sq, int64_t n, unsigned long long *out,
                              hipStream_t st) {
    const int64_t blocks = grid_for(n) < 1024 ? grid_for(n) : 1024;
    hipLaunchKernelGGL(col_max_kernel, dim3((unsigned)blocks), dim3(256), 0, st, col_cnt, col_sq, n, out);
    return hipGetLastError();
}

hipError_t launch_write_records_dev(int vk, int64_t m, const int64_t *row_ptr, const int32_t *col,
                                    const void *vals, const double *b, const RowAux *aux, int64_t stride,
                                    const RowLoc *loc, uint8_t *rec, hipStream_t st) {
    const dim3 grid((unsigned)grid_for(m)), block(256);
    switch (vk) {
        case ASYRK_F64:
            hipLaunchKernelGGL(write_records_kernel<ASYRK_F64>, grid, block, 0, st, m, row_ptr, col,
                               static_cast<const double *>(vals), b, aux, stride, loc, rec);
            break;
        case ASYRK_F32:
            hipLaunchKernelGGL(write_records_kernel<ASYRK_F32>, grid, block, 0, st, m, row_ptr, col,
                               static_cast<const float *>(vals), b, aux, stride, loc, rec);
            break;
        case ASYRK_BF16:
            hipLaunchKernelGGL(write_records_kernel<ASYRK_BF16>, grid, block, 0, st, m, row_ptr, col,
                               static_cast<const uint16_t *>(vals), b, aux, stride, loc, rec);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace asyrk
