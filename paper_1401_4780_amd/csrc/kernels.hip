// gfx950 kernels of the asynchronous randomized Kaczmarz library.
//
// Hot path (sweep_kernel): each group of G lanes is one row worker (Section 3
// of the paper: every worker draws a row, reads x on the row's support without
// locking, forms a_i^T x - b_i and writes every coordinate of supp(a_i) with
// an atomic addition; eq. (2) with step length gamma).  Workers take tickets
// j = t_begin + w, + R, + 2R, ... so R workers are in flight at once.
//
// Memory behaviour:
//   * row records stream from HBM with 16-byte loads, one unit per lane;
//   * x is read with agent-scope relaxed atomic loads (global_load sc1) so a
//     read sees every atomic already performed by any XCD, and written with
//     no-return global_atomic_add_f32/f64; each element of x has a cache line
//     of its own (element c at x[c << xshift]) so that accesses to
//     neighbouring columns do not queue behind each other;
//   * no LDS and no MFMA: there is no dense contraction in this method.
#include "device.h"

namespace asyrk {

template <int VK, int XK, int G>
__global__ __launch_bounds__(256) void sweep_kernel(const SweepArgs a) {
    using X = typename std::conditional<XK == ASYRK_F64, double, float>::type;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t worker = wave * (64 / G) + (lane / G);
    if (worker >= a.R) return;  // whole groups leave together

    X *x = reinterpret_cast<X *>(a.x);
    const X gamma = (X)a.gamma;
    TauAcc acc;
    TauProbe tp{a.tau_ctr, false, 0, 0, 0, 0};
    int64_t it = 0;
    uint32_t mine = 0;
    for (int64_t j = a.t_begin + worker; j < a.t_end; j += a.R, ++it) {
        tp.sample = a.trace != nullptr && it % kTauPeriod == kTauFlush;
        process_ticket<VK, XK, G>(a.rows, x, a.xshift, a.side, j, a.stream_id, a.key0, a.key1, a.uniform,
                                  a.update_one, gamma, gl, a.trace ? &tp : nullptr);
        if (a.trace) {
            if (tp.sample) tau_accumulate(acc, tp.c0, tp.c1, tp.t0, tp.t1);
            ++mine;
            if (it % kTauFlush == kTauFlush - 1) tau_flush_wave(a.tau_ctr, wave, gl, mine);
        }
        if (a.replay) __threadfence();
    }
    if (a.trace) {
        tau_flush_leader(a.tau_ctr, wave, gl, mine);
        tau_store(acc, a.trace, wave, lane);
    }
}

// The same worker loop with the steps of consecutive tickets overlapped
// (LOOP 1, run_tickets_pipelined) or with the records fetched in batches
// (LOOP 2, run_rows_batched): for asynchronous, all-coordinate sweeps.
// TRACE: the instance that samples the staleness.
template <int VK, int XK, int G, bool TRACE, int LOOP>
__global__ __launch_bounds__(256) void sweep_pipe_kernel(const SweepArgs a) {
    using X = typename std::conditional<XK == ASYRK_F64, double, float>::type;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t worker = wave * (64 / G) + (lane / G);
    if (worker >= a.R) return;
    TauAcc acc;
    if constexpr (LOOP == 2)
        run_rows_batched<VK, XK, G, Upl<G>::value, TRACE>(
            a.rows, reinterpret_cast<X *>(a.x), a.xshift, a.side, a.t_begin + worker, a.t_end, a.R, a.uniform,
            (X)a.gamma, gl, SampledPick{(uint32_t)a.rows.m, a.stream_id, a.key0, a.key1}, a.tau_ctr, wave, &acc);
    else
        run_tickets_pipelined<VK, XK, G, Upl<G>::value, TRACE>(a.rows, reinterpret_cast<X *>(a.x), a.xshift, a.side,
                                                               a.t_begin + worker, a.t_end, a.R, a.stream_id, a.key0,
                                                               a.key1, a.uniform, (X)a.gamma, gl, a.tau_ctr, wave, &acc);
    if constexpr (TRACE) tau_store(acc, a.trace, wave, lane);
}

// Without-replacement slice scheme (the paper's experiments): worker w owns
// rows [w L, min(m, (w + 1) L)), L = ceil(m / R), and visits them in a fresh
// keyed permutation every sweep; one launch covers sweeps
// t_begin / m .. t_end / m - 1.
template <int VK, int XK, int G>
__global__ __launch_bounds__(256) void sweep_slices_kernel(const SweepArgs a) {
    using X = typename std::conditional<XK == ASYRK_F64, double, float>::type;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t worker = wave * (64 / G) + (lane / G);
    if (worker >= a.R) return;
    const int64_t m = a.rows.m;
    const int64_t L = (m + a.R - 1) / a.R;
    const int64_t start = worker * L;
    const int64_t Lw = start >= m ? 0 : (m - start < L ? m - start : L);
    X *x = reinterpret_cast<X *>(a.x);
    const X gamma = (X)a.gamma;
    TauAcc acc;
    TauProbe tp{a.tau_ctr, false, 0, 0, 0, 0};
    int64_t it = 0;
    uint32_t mine = 0;
    for (int64_t sw = a.t_begin / m; sw < a.t_end / m && Lw > 0; ++sw) {
        const U4 u = philox4x32_10((uint32_t)((uint64_t)sw & 0xffffffffu), (uint32_t)((uint64_t)sw >> 32),
                                   (uint32_t)worker, 0x5C4E3D2Bu, a.key0, a.key1);
        for (int64_t k = 0; k < Lw; ++k, ++it) {
            const uint32_t i = (uint32_t)(start + slice_perm((uint32_t)k, (uint32_t)Lw, u));
            tp.sample = a.trace != nullptr && it % kTauPeriod == kTauFlush;
            process_ticket<VK, XK, G, Upl<G>::value, false>(a.rows, x, a.xshift, a.side, 0, 0u, 0u, 0u, 1, 0, gamma,
                                                             gl, a.trace ? &tp : nullptr, i);
            if (a.trace) {
                if (tp.sample) tau_accumulate(acc, tp.c0, tp.c1, tp.t0, tp.t1);
                ++mine;
                if (it % kTauFlush == kTauFlush - 1) tau_flush_wave(a.tau_ctr, wave, gl, mine);
            }
            if (a.replay) __threadfence();
        }
    }
    if (a.trace) {
        tau_flush_leader(a.tau_ctr, wave, gl, mine);
        tau_store(acc, a.trace, wave, lane);
    }
}

// The same slice walks, each fed to the software-pipelined worker loop as a
// stream of tickets (asynchronous, all-coordinate sweeps).
template <int VK, int XK, int G, bool TRACE, int LOOP>
__global__ __launch_bounds__(256) void sweep_slices_pipe_kernel(const SweepArgs a) {
    using X = typename std::conditional<XK == ASYRK_F64, double, float>::type;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t worker = wave * (64 / G) + (lane / G);
    if (worker >= a.R) return;
    const int64_t m = a.rows.m;
    const int64_t L = (m + a.R - 1) / a.R;
    const int64_t start = worker * L;
    const int64_t Lw = start >= m ? 0 : (m - start < L ? m - start : L);
    TauAcc acc;
    const SlicePick walk{start, a.t_begin / m, (uint32_t)Lw, (uint32_t)worker, a.key0, a.key1};
    if (Lw > 0) {
        if constexpr (LOOP == 2)
            run_rows_batched<VK, XK, G, Upl<G>::value, TRACE>(a.rows, reinterpret_cast<X *>(a.x), a.xshift, a.side,
                                                              0, (a.t_end - a.t_begin) / m * Lw, 1, 1, (X)a.gamma,
                                                              gl, walk, a.tau_ctr, wave, &acc);
        else
            run_rows_pipelined<VK, XK, G, Upl<G>::value, TRACE>(a.rows, reinterpret_cast<X *>(a.x), a.xshift, a.side,
                                                                0, (a.t_end - a.t_begin) / m * Lw, 1, 1, (X)a.gamma,
                                                                gl, walk, a.tau_ctr, wave, &acc);
    }
    if constexpr (TRACE) tau_store(acc, a.trace, wave, lane);
}

// The batched loop of a wave-wide worker split over two waves (a fetch wave
// and a compute wave, run_rows_split): one workgroup per worker, two LDS
// batch buffers.  Sampled rows, or (SLICES) the worker's slice walk.
template <int VK, int XK, bool TRACE, bool SLICES>
__global__ __launch_bounds__(128) void sweep_split_kernel(const SweepArgs a) {
    using X = typename std::conditional<XK == ASYRK_F64, double, float>::type;
    constexpr int B = SplitBatch<VK>::value;
    __shared__ Unit<VK> lu[2][B][64];
    __shared__ SplitMeta<XK> lm[2][B];
    // a scalar: each wave branches to its role as a whole and never runs the
    // other role's code (whose barriers it would otherwise pass with no
    // lanes active: s_barrier counts waves, not lanes)
    const int role = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int64_t worker = blockIdx.x;
    if (worker >= a.R) return;  // the whole workgroup
    TauAcc acc;
    if constexpr (SLICES) {
        const int64_t m = a.rows.m;
        const int64_t L = (m + a.R - 1) / a.R;
        const int64_t start = worker * L;
        const int64_t Lw = start >= m ? 0 : (m - start < L ? m - start : L);
        if (Lw > 0) {
            const SlicePick walk{start, a.t_begin / m, (uint32_t)Lw, (uint32_t)worker, a.key0, a.key1};
            run_rows_split<VK, XK, TRACE>(a.rows, reinterpret_cast<X *>(a.x), a.xshift, a.side, 0,
                                          (a.t_end - a.t_begin) / m * Lw, 1, 1, (X)a.gamma, role, lane, walk, lu,
                                          lm, a.tau_ctr, worker, &acc);
        }
    } else {
        run_rows_split<VK, XK, TRACE>(a.rows, reinterpret_cast<X *>(a.x), a.xshift, a.side, a.t_begin + worker,
                                      a.t_end, a.R, a.uniform, (X)a.gamma, role, lane,
                                      SampledPick{(uint32_t)a.rows.m, a.stream_id, a.key0, a.key1}, lu, lm,
                                      a.tau_ctr, worker, &acc);
    }
    if constexpr (TRACE) {
        if (role == 0) tau_store(acc, a.trace, worker, lane);
    }
}

// The batched loop with G = 64 runs split over two waves up to this many
// workers (one workgroup of two waves per worker).
constexpr int64_t kSplitMaxR = 512;

template <int VK, int XK, bool SLICES>
static hipError_t launch_split(const SweepArgs &a, hipStream_t st) {
    if (a.trace)
        hipLaunchKernelGGL((sweep_split_kernel<VK, XK, true, SLICES>), dim3(a.R), dim3(128), 0, st, a);
    else
        hipLaunchKernelGGL((sweep_split_kernel<VK, XK, false, SLICES>), dim3(a.R), dim3(128), 0, st, a);
    return hipGetLastError();
}

// Calls f(std::integral_constant<int, G>) for a lane-group width G in
// {1, 2, 4, ..., 64}, then returns the launch status.
template <class F>
static hipError_t dispatch_lanes(int G, F &&f) {
    switch (G) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 8: f(std::integral_constant<int, 8>{}); break;
        case 16: f(std::integral_constant<int, 16>{}); break;
        case 32: f(std::integral_constant<int, 32>{}); break;
        case 64: f(std::integral_constant<int, 64>{}); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The pipelined loop serves the latency-bound regime (few workers): one
// wave per block spreads those workers over as many CUs as there are waves
// instead of packing four waves onto each CU's memory pipeline.
static void sweep_geometry(const SweepArgs &a, int G, int64_t *grid, int *block) {
    const int64_t threads = a.R * G;
    *block = a.pipe ? 64 : (threads < 256 ? (int)(((threads + 63) / 64) * 64) : 256);
    *grid = (threads + *block - 1) / *block;
}

template <int VK, int XK>
static hipError_t launch_slices_vk(int G, const SweepArgs &a, hipStream_t st) {
    int64_t grid;
    int block;
    sweep_geometry(a, G, &grid, &block);
    if (a.pipe == 2 && G == 64 && a.R <= kSplitMaxR) return launch_split<VK, XK, true>(a, st);
    if (a.pipe == 2 && a.trace)
        return dispatch_lanes(G, [&](auto g) {
            hipLaunchKernelGGL((sweep_slices_pipe_kernel<VK, XK, decltype(g)::value, true, 2>), dim3(grid), dim3(block), 0, st, a);
        });
    if (a.pipe == 2)
        return dispatch_lanes(G, [&](auto g) {
            hipLaunchKernelGGL((sweep_slices_pipe_kernel<VK, XK, decltype(g)::value, false, 2>), dim3(grid), dim3(block), 0, st, a);
        });
    if (a.pipe && a.trace)
        return dispatch_lanes(G, [&](auto g) {
            hipLaunchKernelGGL((sweep_slices_pipe_kernel<VK, XK, decltype(g)::value, true, 1>), dim3(grid), dim3(block), 0, st, a);
        });
    if (a.pipe)
        return dispatch_lanes(G, [&](auto g) {
            hipLaunchKernelGGL((sweep_slices_pipe_kernel<VK, XK, decltype(g)::value, false, 1>), dim3(grid), dim3(block), 0, st, a);
        });
    return dispatch_lanes(G, [&](auto g) {
        hipLaunchKernelGGL((sweep_slices_kernel<VK, XK, decltype(g)::value>), dim3(grid), dim3(block), 0, st, a);
    });
}

hipError_t launch_sweep_slices(int vk, int xk, int G, const SweepArgs &a, hipStream_t st) {
    if (xk == ASYRK_F32) {
        switch (vk) {
            case ASYRK_F32: return launch_slices_vk<ASYRK_F32, ASYRK_F32>(G, a, st);
            case ASYRK_BF16: return launch_slices_vk<ASYRK_BF16, ASYRK_F32>(G, a, st);
        }
    } else if (xk == ASYRK_F64) {
        switch (vk) {
            case ASYRK_F32: return launch_slices_vk<ASYRK_F32, ASYRK_F64>(G, a, st);
            case ASYRK_BF16: return launch_slices_vk<ASYRK_BF16, ASYRK_F64>(G, a, st);
            case ASYRK_F64: return launch_slices_vk<ASYRK_F64, ASYRK_F64>(G, a, st);
        }
    }
    return hipErrorInvalidValue;
}

template <int VK, int XK>
static hipError_t launch_sweep_vk(int G, const SweepArgs &a, hipStream_t st) {
    int64_t grid;
    int block;
    sweep_geometry(a, G, &grid, &block);
    if (a.pipe == 2 && G == 64 && a.R <= kSplitMaxR) return launch_split<VK, XK, false>(a, st);
    if (a.pipe == 2 && a.trace)
        return dispatch_lanes(G, [&](auto g) {
            hipLaunchKernelGGL((sweep_pipe_kernel<VK, XK, decltype(g)::value, true, 2>), dim3(grid), dim3(block), 0, st, a);
        });
    if (a.pipe == 2)
        return dispatch_lanes(G, [&](auto g) {
            hipLaunchKernelGGL((sweep_pipe_kernel<VK, XK, decltype(g)::value, false, 2>), dim3(grid), dim3(block), 0, st, a);
        });
    if (a.pipe && a.trace)
        return dispatch_lanes(G, [&](auto g) {
            hipLaunchKernelGGL((sweep_pipe_kernel<VK, XK, decltype(g)::value, true, 1>), dim3(grid), dim3(block), 0, st, a);
        });
    if (a.pipe)
        return dispatch_lanes(G, [&](auto g) {
            hipLaunchKernelGGL((sweep_pipe_kernel<VK, XK, decltype(g)::value, false, 1>), dim3(grid), dim3(block), 0, st, a);
        });
    return dispatch_lanes(G, [&](auto g) {
        hipLaunchKernelGGL((sweep_kernel<VK, XK, decltype(g)::value>), dim3(grid), dim3(block), 0, st, a);
    });
}

hipError_t launch_sweep(int vk, int xk, int G, const SweepArgs &a, hipStream_t st) {
    if (xk == ASYRK_F32) {
        switch (vk) {
            case ASYRK_F32: return launch_sweep_vk<ASYRK_F32, ASYRK_F32>(G, a, st);
            case ASYRK_BF16: return launch_sweep_vk<ASYRK_BF16, ASYRK_F32>(G, a, st);
        }
    } else if (xk == ASYRK_F64) {
        switch (vk) {
            case ASYRK_F32: return launch_sweep_vk<ASYRK_F32, ASYRK_F64>(G, a, st);
            case ASYRK_BF16: return launch_sweep_vk<ASYRK_BF16, ASYRK_F64>(G, a, st);
            case ASYRK_F64: return launch_sweep_vk<ASYRK_F64, ASYRK_F64>(G, a, st);
        }
    }
    return hipErrorInvalidValue;
}

// side[i] = {b_i, 1/w_i} in FP64, w_i = ||a_i||^2 from the stored values
// (summed in record order; FP64 iterate over FP32/BF16 records).
template <int VK>
__global__ __launch_bounds__(256) void build_side_kernel(const Rows rows, const double *b64, double2 *side) {
    using T = VT<VK>;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows.m; i += stride) {
        const uint8_t *rec;
        int nnz;
        locate(rows, (uint32_t)i, rec, nnz);
        double w = 0.0;
        for (int k = 0; k < nnz; ++k) {
            int c;
            typename T::x_t v;
            load_entry<VK>(rec, k, c, v);
            w = __dadd_rn(w, __dmul_rn((double)v, (double)v));
        }
        side[i] = make_double2(b64[i], 1.0 / w);
    }
}

hipError_t launch_build_side(int vk, const Rows &rows, const double *b64, double2 *side, hipStream_t st) {
    const int grid = (int)((rows.m + 255) / 256 < 8192 ? (rows.m + 255) / 256 : 8192);
    switch (vk) {
        case ASYRK_F32: hipLaunchKernelGGL(build_side_kernel<ASYRK_F32>, dim3(grid), dim3(256), 0, st, rows, b64, side); break;
        case ASYRK_BF16: hipLaunchKernelGGL(build_side_kernel<ASYRK_BF16>, dim3(grid), dim3(256), 0, st, rows, b64, side); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- reductions

// Sum of one value per thread into partials[blockIdx.x], fixed order.
__device__ __forceinline__ void block_sum_store(double v, double *partials) {
    __shared__ double wsum[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) wsum[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += wsum[k];
        partials[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void finish_sum_kernel(const double *partials, int nparts, double *out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) s += partials[k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

hipError_t launch_finish_sum(const double *partials, int nparts, double *out, hipStream_t st) {
    hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(256), 0, st, partials, nparts, out);
    return hipGetLastError();
}

template <class XI>
__global__ __launch_bounds__(256) void sumsq_diff_kernel(const XI *x, int xsh, const double *xr, int64_t n,
                                                          double *partials) {
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
        const double d = (double)x[c << xsh] - (xr ? xr[c] : 0.0);
        s += d * d;
    }
    block_sum_store(s, partials);
}

hipError_t launch_sumsq_diff(const void *x, int x_is_f32, int xsh, const double *xr, int64_t n,
                             double *partials, int nblocks, hipStream_t st) {
    if (x_is_f32)
        hipLaunchKernelGGL(sumsq_diff_kernel<float>, dim3(nblocks), dim3(256), 0, st,
                           (const float *)x, xsh, xr, n, partials);
    else
        hipLaunchKernelGGL(sumsq_diff_kernel<double>, dim3(nblocks), dim3(256), 0, st,
                           (const double *)x, xsh, xr, n, partials);
    return hipGetLastError();
}

// ---------------------------------------------------------------- residual (FP64)
// r_i = b_i - sum_k v_k x_{c_k}, stored values promoted exactly to FP64
// (b64 == nullptr: r = -A x; rhs_from_rec: b_i is the record header's b,
// i.e. the right-hand side the sweeps currently solve for).
// One group of 4 lanes per row, rows in order (coalesced record stream).
template <int VK, class XI>
__global__ __launch_bounds__(256) void residual_kernel(const Rows rows, const double *b64, const XI *x, int xsh,
                                                        double *r_out, int write_rec_b, double *partials,
                                                        int rhs_from_rec) {
    using T = VT<VK>;
    constexpr int G = 4;
    const int gl = threadIdx.x & (G - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    double sq = 0.0;
    for (int64_t i = grp; i < rows.m; i += ngrp) {
        const uint8_t *rec;
        int nnz;
        locate(rows, (uint32_t)i, rec, nnz);
        const int nunits = (nnz + T::U - 1) / T::U;
        double acc = 0.0;
        for (int uu = gl; uu < nunits; uu += G) {
            Unit<VK> un;
            un.load(rec + T::HB + (int64_t)uu * T::UB);
#pragma unroll
            for (int e = 0; e < T::U; ++e)
                if (uu * T::U + e < nnz) acc = fma((double)un.v[e], (double)x[(int64_t)un.c[e] << xsh], acc);
        }
        acc = group_sum<G>(acc);
        double bi = b64 ? b64[i] : 0.0;
        if (rhs_from_rec) bi = (double)load_hdr<VK>(rec).b;
        const double r = bi - acc;
        if (gl == 0) {
            if (r_out) r_out[i] = r;
            if (write_rec_b) {
                using HB = typename T::hdr_t;
                reinterpret_cast<HB *>(const_cast<uint8_t *>(rec))->b = (decltype(HB::b))r;
            }
            sq += r * r;
        }
    }
    block_sum_store(sq, partials);
}

template <int VK>
static hipError_t launch_residual_vk(const Rows &rows, const double *b64, const void *x, int x_is_f32, int xsh,
                                     double *r_out, int write_rec_b, double *partials, int nblocks,
                                     int rhs_from_rec, hipStream_t st) {
    if (x_is_f32)
        hipLaunchKernelGGL((residual_kernel<VK, float>), dim3(nblocks), dim3(256), 0, st, rows, b64,
                           (const float *)x, xsh, r_out, write_rec_b, partials, rhs_from_rec);
    else
        hipLaunchKernelGGL((residual_kernel<VK, double>), dim3(nblocks), dim3(256), 0, st, rows, b64,
                           (const double *)x, xsh, r_out, write_rec_b, partials, rhs_from_rec);
    return hipGetLastError();
}

hipError_t launch_residual(int vk, const Rows &rows, const double *b64, const void *x, int x_is_f32, int xsh,
                           double *r_out, int write_rec_b, double *partials, int nblocks,
                           hipStream_t st, int rhs_from_rec) {
    switch (vk) {
        case ASYRK_F32: return launch_residual_vk<ASYRK_F32>(rows, b64, x, x_is_f32, xsh, r_out, write_rec_b, partials, nblocks, rhs_from_rec, st);
        case ASYRK_BF16: return launch_residual_vk<ASYRK_BF16>(rows, b64, x, x_is_f32, xsh, r_out, write_rec_b, partials, nblocks, rhs_from_rec, st);
        case ASYRK_F64: return launch_residual_vk<ASYRK_F64>(rows, b64, x, x_is_f32, xsh, r_out, write_rec_b, partials, nblocks, rhs_from_rec, st);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- record b

template <int VK>
__global__ __launch_bounds__(256) void set_rec_b_kernel(const Rows rows, const double *b64) {
    using HB = typename VT<VK>::hdr_t;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows.m; i += stride) {
        const uint8_t *rec;
        int nnz;
        locate(rows, (uint32_t)i, rec, nnz);
        reinterpret_cast<HB *>(const_cast<uint8_t *>(rec))->b = (decltype(HB::b))b64[i];
    }
}

hipError_t launch_set_rec_b(int vk, const Rows &rows, const double *b64, hipStream_t st) {
    const int grid = (int)((rows.m + 255) / 256 < 8192 ? (rows.m + 255) / 256 : 8192);
    switch (vk) {
        case ASYRK_F32: hipLaunchKernelGGL(set_rec_b_kernel<ASYRK_F32>, dim3(grid), dim3(256), 0, st, rows, b64); break;
        case ASYRK_BF16: hipLaunchKernelGGL(set_rec_b_kernel<ASYRK_BF16>, dim3(grid), dim3(256), 0, st, rows, b64); break;
        case ASYRK_F64: hipLaunchKernelGGL(set_rec_b_kernel<ASYRK_F64>, dim3(grid), dim3(256), 0, st, rows, b64); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- vectors

template <class XO>
__global__ __launch_bounds__(256) void cast_to_iter_kernel(const double *x64, XO *xo, int xsh, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) xo[c << xsh] = (XO)x64[c];
}

template <class XI>
__global__ __launch_bounds__(256) void iter_to_f64_kernel(const XI *xi, int xsh, double *x64, int64_t n, int acc) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride)
        x64[c] = acc ? x64[c] + (double)xi[c << xsh] : (double)xi[c << xsh];
}

static int vec_grid(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (int)(g < 4096 ? (g < 1 ? 1 : g) : 4096);
}

hipError_t launch_cast_to_iter(const double *x64, void *xit, int xit_is_f32, int xsh, int64_t n, hipStream_t st) {
    if (xit_is_f32)
        hipLaunchKernelGGL(cast_to_iter_kernel<float>, dim3(vec_grid(n)), dim3(256), 0, st, x64, (float *)xit, xsh, n);
    else
        hipLaunchKernelGGL(cast_to_iter_kernel<double>, dim3(vec_grid(n)), dim3(256), 0, st, x64, (double *)xit, xsh, n);
    return hipGetLastError();
}

hipError_t launch_iter_to_f64(const void *xit, int xit_is_f32, int xsh, double *x64, int64_t n, int accumulate,
                              hipStream_t st) {
    if (xit_is_f32)
        hipLaunchKernelGGL(iter_to_f64_kernel<float>, dim3(vec_grid(n)), dim3(256), 0, st, (const float *)xit, xsh, x64, n, accumulate);
    else
        hipLaunchKernelGGL(iter_to_f64_kernel<double>, dim3(vec_grid(n)), dim3(256), 0, st, (const double *)xit, xsh, x64, n, accumulate);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void zero_kernel(uint32_t *p, int64_t words) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < words; c += stride) p[c] = 0u;
}

hipError_t launch_zero(void *p, int64_t bytes, hipStream_t st) {
    const int64_t words = bytes / 4;
    hipLaunchKernelGGL(zero_kernel, dim3(vec_grid(words)), dim3(256), 0, st, (uint32_t *)p, words);
    return hipGetLastError();
}

// ---------------------------------------------------------------- power iteration pieces

// z += A^T y: row i adds y_i * a_i into z (FP64 atomics).
template <int VK>
__global__ __launch_bounds__(256) void scatter_rows_kernel(const Rows rows, const double *y, double *z) {
    using T = VT<VK>;
    constexpr int G = 4;
    const int gl = threadIdx.x & (G - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    for (int64_t i = grp; i < rows.m; i += ngrp) {
        const uint8_t *rec;
        int nnz;
        locate(rows, (uint32_t)i, rec, nnz);
        const int nunits = (nnz + T::U - 1) / T::U;
        const double yi = y[i];
        for (int uu = gl; uu < nunits; uu += G) {
            Unit<VK> un;
            un.load(rec + T::HB + (int64_t)uu * T::UB);
#pragma unroll
            for (int e = 0; e < T::U; ++e)
                if (uu * T::U + e < nnz) unsafeAtomicAdd(z + un.c[e], yi * (double)un.v[e]);
        }
    }
}

hipError_t launch_scatter_rows(int vk, const Rows &rows, const double *y, double *z, hipStream_t st) {
    const int grid = kResidualBlocks;
    switch (vk) {
        case ASYRK_F32: hipLaunchKernelGGL(scatter_rows_kernel<ASYRK_F32>, dim3(grid), dim3(256), 0, st, rows, y, z); break;
        case ASYRK_BF16: hipLaunchKernelGGL(scatter_rows_kernel<ASYRK_BF16>, dim3(grid), dim3(256), 0, st, rows, y, z); break;
        case ASYRK_F64: hipLaunchKernelGGL(scatter_rows_kernel<ASYRK_F64>, dim3(grid), dim3(256), 0, st, rows, y, z); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void scale_kernel(double *v, int64_t n, const double *norm2) {
    const double s = 1.0 / sqrt(norm2[0]);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) v[c] *= s;
}

hipError_t launch_scale(double *v, int64_t n, const double *norm2, hipStream_t st) {
    hipLaunchKernelGGL(scale_kernel, dim3(vec_grid(n)), dim3(256), 0, st, v, n, norm2);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void divide_kernel(const double *z, double d, double *out, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) out[c] = z[c] / d;
}

hipError_t launch_divide(const double *z, double d, double *out, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(divide_kernel, dim3(vec_grid(n)), dim3(256), 0, st, z, d, out, n);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void random_fill_kernel(double *v, int64_t n, uint32_t k0, uint32_t k1) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
        const U4 u = draw(c, 0xA5A5A5A5u, k0, k1);
        v[c] = ((double)u.a + 0.5) * (1.0 / 4294967296.0) - 0.5;
    }
}

hipError_t launch_random_fill(double *v, int64_t n, uint32_t k0, uint32_t k1, hipStream_t st) {
    hipLaunchKernelGGL(random_fill_kernel, dim3(vec_grid(n)), dim3(256), 0, st, v, n, k0, k1);
    return hipGetLastError();
}

// ---------------------------------------------------------------- sampler exposure
// The exact draw the sweep makes for each ticket, written out for checking.

template <int VK>
__global__ __launch_bounds__(256) void sample_rows_kernel(const Rows rows, int64_t ticket0, int64_t count,
                                                           uint32_t k0, uint32_t k1, uint32_t stream_id,
                                                           int uniform, int32_t *rows_out, int32_t *coords_out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += stride) {
        const U4 u = draw(ticket0 + q, stream_id, k0, k1);
        uint32_t i = bucket_of(u.a, u.b, (uint32_t)rows.m);
        const uint8_t *rec;
        int nnz;
        locate(rows, i, rec, nnz);
        if (!uniform) {
            const typename VT<VK>::hdr_t h = load_hdr<VK>(rec);
            if (!(u.c < h.thresh)) {
                i = (uint32_t)h.alias;
                locate(rows, i, rec, nnz);
            }
        }
        rows_out[q] = (int32_t)i;
        if (coords_out) coords_out[q] = (int32_t)(((uint64_t)u.d * (uint64_t)nnz) >> 32);
    }
}

hipError_t launch_sample_rows(int vk, const Rows &rows, int64_t ticket0, int64_t count, uint32_t k0,
                              uint32_t k1, uint32_t stream_id, int uniform, int32_t *rows_out,
                              int32_t *coords_out, hipStream_t st) {
    const int grid = vec_grid(count);
    switch (vk) {
        case ASYRK_F32: hipLaunchKernelGGL(sample_rows_kernel<ASYRK_F32>, dim3(grid), dim3(256), 0, st, rows, ticket0, count, k0, k1, stream_id, uniform, rows_out, coords_out); break;
        case ASYRK_BF16: hipLaunchKernelGGL(sample_rows_kernel<ASYRK_BF16>, dim3(grid), dim3(256), 0, st, rows, ticket0, count, k0, k1, stream_id, uniform, rows_out, coords_out); break;
        case ASYRK_F64: hipLaunchKernelGGL(sample_rows_kernel<ASYRK_F64>, dim3(grid), dim3(256), 0, st, rows, ticket0, count, k0, k1, stream_id, uniform, rows_out, coords_out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- device ceilings

__global__ __launch_bounds__(256) void probe_copy_kernel(const float4 *src, float4 *dst, int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n4; c += stride) dst[c] = src[c];
}

// Random accesses to a table of n elements: kind 0 agent-coherent loads, kind 1
// no-return atomic adds.  Addresses come from a counter hash (no index stream).
template <class X>
__global__ __launch_bounds__(256) void probe_scatter_kernel(X *tab, uint32_t n, int64_t count, int kind,
                                                             X *sink) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    X acc = (X)0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += stride) {
        uint32_t h = (uint32_t)q * 0x9E3779B1u;
        h ^= h >> 15;
        h *= 0x2C1B3C6Du;
        h ^= h >> 12;
        const uint32_t c = (uint32_t)(((uint64_t)h * n) >> 32);
        if (kind == 0)
            acc += load_agent(tab + c);
        else
            unsafeAtomicAdd(tab + c, (X)1);
    }
    if (kind == 0 && acc == (X)-12345.0) sink[0] = acc;  // keeps the loads alive
}

hipError_t probe_copy(int64_t bytes, int iters, double *gbps) {
    const int64_t n4 = bytes / 16;
    float4 *src = nullptr, *dst = nullptr;
    hipEvent_t e0, e1;
    hipError_t err = hipMalloc(&src, n4 * 16);
    if (err != hipSuccess) return err;
    err = hipMalloc(&dst, n4 * 16);
    if (err != hipSuccess) { (void)hipFree(src); return err; }
    (void)hipMemset(src, 0, n4 * 16);
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int grid = 256 * 32;
    hipLaunchKernelGGL(probe_copy_kernel, dim3(grid), dim3(256), 0, 0, src, dst, n4);
    (void)hipEventRecord(e0, 0);
    for (int it = 0; it < iters; ++it)
        hipLaunchKernelGGL(probe_copy_kernel, dim3(grid), dim3(256), 0, 0, src, dst, n4);
    (void)hipEventRecord(e1, 0);
    err = hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *gbps = 2.0 * (double)n4 * 16.0 * iters / (ms * 1e-3) / 1e9;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(src);
    (void)hipFree(dst);
    return err == hipSuccess ? hipGetLastError() : err;
}

hipError_t probe_scatter(int64_t n, int64_t count, int dtype, int kind, int iters, double *per_s) {
    const size_t esz = dtype == ASYRK_F64 ? 8 : 4;
    void *tab = nullptr;
    hipEvent_t e0, e1;
    hipError_t err = hipMalloc(&tab, (size_t)n * esz + 64);
    if (err != hipSuccess) return err;
    (void)hipMemset(tab, 0, (size_t)n * esz + 64);
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int grid = 256 * 16;
    auto launch = [&]() {
        if (dtype == ASYRK_F64)
            hipLaunchKernelGGL(probe_scatter_kernel<double>, dim3(grid), dim3(256), 0, 0, (double *)tab,
                               (uint32_t)n, count, kind, (double *)tab + n);
        else
            hipLaunchKernelGGL(probe_scatter_kernel<float>, dim3(grid), dim3(256), 0, 0, (float *)tab,
                               (uint32_t)n, count, kind, (float *)tab + n);
    };
    launch();
    (void)hipEventRecord(e0, 0);
    for (int it = 0; it < iters; ++it) launch();
    (void)hipEventRecord(e1, 0);
    err = hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *per_s = (double)count * iters / (ms * 1e-3);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(tab);
    return err == hipSuccess ? hipGetLastError() : err;
}

}  // namespace asyrk
