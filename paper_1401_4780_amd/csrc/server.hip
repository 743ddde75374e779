// Serving engine: many independent consistent systems solved concurrently on
// one GPU with continuous batching.
//
//   submit()   (any thread)  validate + pack a request on the caller's thread,
//                            queue it.
//   progress() (one thread)  serves one of two groups of active systems,
//                            the groups taking turns, so that one group's
//                            round computes while the host serves the other:
//       collect the group's previous round, and retire requests whose FP64
//               relative residual met their tolerance (or whose round budget
//               ran out): copy x out, free its memory;
//       admit   queued requests while the worker budget and the device-
//               memory budget allow (first-fit arena: no device allocation or
//               free in the loop); their uploads run on a copy stream, and a
//               request joins a group's round once its upload has finished
//               (waited for only when the GPU has nothing else to do);
//       run     the group's round, one packed launch per phase over its
//               systems: zero d -> asynchronous sweeps on A d = r (FP32
//               values, FP64 correction d and FP64 atomics) -> x += d (FP64)
//               -> r = b - A x (FP64, written to the per-row side records as
//               the next round's right-hand side) -> per-system ||r||^2.
//               The four launches are captured per group and sweep variant in
//               a hipGraph (fixed grids; kernels read the group's slot table).
//   poll()     (any thread)  fetch a finished request's x and statistics.
//
// Each system runs R_s row workers with R_s bounded by its own Corollary 1
// limit (tau + 1 <= ||A||_F^2 / (2 e lambda)), so small systems take few
// workers and the GPU is filled by packing many systems into one launch.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "device.h"
#include "setup.h"

using namespace asyrk;

namespace {

constexpr int kVecBlocks = 2048;     // grid of the flat vector/residual kernels
// Candidate lane widths of the plain and the pipelined sweep, and the number
// of load buckets the online choice keeps apart.
constexpr int kLaneCands[2][4] = {{4, 8, 0, 0}, {4, 8, 16, 32}};
constexpr int kNumCands[2] = {2, 4};
constexpr int kBuckets = 4;

struct SlotDesc {
    Rows rows;
    double *b64;
    double *x64;
    double *d;        // correction, FP64 (FP64 atomics are the faster ones), element c at d[c << xshift]
    double2 *side;    // per row {r_i, 1/||a_i||^2}: the correction system's right-hand side
    int64_t n;
    int64_t R;        // row workers of this system
    int64_t w_off;    // first global worker
    int64_t row_off;  // first global row
    int64_t col_off;  // first global column
    int64_t t_begin, t_end;
    uint32_t key0, key1;
    double gamma;
    int32_t xshift;   // log2 of the correction's element stride
    int32_t pad;
};

struct TableHead {
    int32_t nact;
    int32_t pad;
    int64_t total_workers, total_rows, total_cols;
};

// binary search: last slot s with off(s) <= q
template <class F>
__device__ __forceinline__ int find_slot(int nact, int64_t q, F off) {
    int lo = 0, hi = nact - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off(mid) <= q)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void srv_zero_kernel(const TableHead *th, const SlotDesc *sl, double *norm2) {
    const int nact = th->nact;
    const int64_t total = th->total_cols;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < nact) norm2[tid] = 0.0;
    for (int64_t q = tid; q < total; q += stride) {
        const int s = find_slot(nact, q, [&](int k) { return sl[k].col_off; });
        sl[s].d[(q - sl[s].col_off) << sl[s].xshift] = 0.0;
    }
}

// G lanes per row with 16 / G units per lane (one for G = 32, half of the
// lanes idle on the longest rows): rows of up to 64 FP32 entries
// stay in registers.  PIPE: the pipelined worker loop, for rounds with few
// workers (latency-bound); the plain loop saturates the atomic unit better
// when many are active.
template <int G, bool PIPE, bool SLICES = false>
__device__ __forceinline__ void srv_sweep_body(const TableHead *th, const SlotDesc *sl) {
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t worker = wave * (64 / G) + (lane / G);
    if (worker >= th->total_workers) return;
    const int s = find_slot(th->nact, worker, [&](int k) { return sl[k].w_off; });
    const SlotDesc d = sl[s];  // a copy: the scatter cannot be taken to alias it
    const int64_t w = worker - d.w_off;
    if constexpr (PIPE && SLICES) {
        // the slice walk (see srv_sweep_slices_kernel) as a ticket stream
        const int64_t m = d.rows.m;
        const int64_t L = (m + d.R - 1) / d.R;
        const int64_t start = w * L;
        const int64_t Lw = start >= m ? 0 : (m - start < L ? m - start : L);
        if (Lw == 0) return;
        run_rows_pipelined<ASYRK_F32, ASYRK_F64, G, (G < 16 ? 16 / G : 1)>(
            d.rows, d.d, d.xshift, d.side, 0, (d.t_end - d.t_begin) / m * Lw, 1, 1, d.gamma, gl,
            SlicePick{start, d.t_begin / m, (uint32_t)Lw, (uint32_t)w, d.key0, d.key1});
    } else if constexpr (PIPE) {
        run_tickets_pipelined<ASYRK_F32, ASYRK_F64, G, (G < 16 ? 16 / G : 1)>(d.rows, d.d, d.xshift, d.side, d.t_begin + w, d.t_end, d.R,
                                                               0u, d.key0, d.key1, 0, d.gamma, gl);
    } else {
        for (int64_t j = d.t_begin + w; j < d.t_end; j += d.R)
            process_ticket<ASYRK_F32, ASYRK_F64, G, (G < 16 ? 16 / G : 1)>(d.rows, d.d, d.xshift, d.side, j, 0u, d.key0, d.key1, 0, 0,
                                                             d.gamma, gl, 0);
    }
}

// Plain loop: four waves per SIMD keep the default 65536 workers (x 4 lanes)
// resident at once.
template <int G>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void srv_sweep_kernel(const TableHead *th, const SlotDesc *sl) {
    srv_sweep_body<G, false>(th, sl);
}

// Plain loop without replacement (the slice scheme of the paper's
// experiments): worker w of a system owns its rows [w L, min(m, (w + 1) L)),
// L = ceil(m / R), and visits them in a fresh keyed permutation every sweep
// of the round; a round's tickets cover whole sweeps.
template <int G>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void srv_sweep_slices_kernel(
    const TableHead *th, const SlotDesc *sl) {
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t worker = wave * (64 / G) + (lane / G);
    if (worker >= th->total_workers) return;
    const int s = find_slot(th->nact, worker, [&](int k) { return sl[k].w_off; });
    const SlotDesc d = sl[s];
    const int64_t w = worker - d.w_off;
    const int64_t m = d.rows.m;
    const int64_t L = (m + d.R - 1) / d.R;
    const int64_t start = w * L;
    const int64_t Lw = start >= m ? 0 : (m - start < L ? m - start : L);
    for (int64_t sw = d.t_begin / m; sw < d.t_end / m; ++sw) {
        const U4 u = philox4x32_10((uint32_t)((uint64_t)sw & 0xffffffffu), (uint32_t)((uint64_t)sw >> 32),
                                   (uint32_t)w, 0x5C4E3D2Bu, d.key0, d.key1);
        for (int64_t k = 0; k < Lw; ++k) {
            const uint32_t i = (uint32_t)(start + slice_perm((uint32_t)k, (uint32_t)Lw, u));
            process_ticket<ASYRK_F32, ASYRK_F64, G, (G < 16 ? 16 / G : 1), false>(
                d.rows, d.d, d.xshift, d.side, 0, 0u, 0u, 0u, 1, 0, d.gamma, gl, 0, i);
        }
    }
}

// Pipelined loop: its rounds hold at most a few thousand workers, so it may
// use the registers of two tickets without an occupancy bound.
template <int G, bool SLICES>
__global__ __launch_bounds__(256) void srv_sweep_pipe_kernel(const TableHead *th, const SlotDesc *sl) {
    srv_sweep_body<G, true, SLICES>(th, sl);
}

__global__ __launch_bounds__(256) void srv_axpy_kernel(const TableHead *th, const SlotDesc *sl) {
    const int nact = th->nact;
    const int64_t total = th->total_cols;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
        const int s = find_slot(nact, q, [&](int k) { return sl[k].col_off; });
        const int64_t c = q - sl[s].col_off;
        sl[s].x64[c] += sl[s].d[c << sl[s].xshift];
    }
}

// r = b - A x64 in FP64 (4 lanes per row); r becomes the side record's
// right-hand side for the next round; ||r||^2 accumulates per system.
__global__ __launch_bounds__(256) void srv_residual_kernel(const TableHead *th, const SlotDesc *sl, double *norm2) {
    using T = VT<ASYRK_F32>;
    constexpr int G = 4;
    const int nact = th->nact;
    const int64_t total = th->total_rows;
    const int gl = threadIdx.x & (G - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    // every wave runs the same trip count so the wave-wide sums below see all lanes
    const int64_t wave0 = (grp / (64 / G)) * (64 / G);
    for (int64_t qb = wave0; qb < total; qb += ngrp) {
        const int64_t q = qb + (grp - wave0);
        const bool live = q < total;
        int s = -1;
        double r2 = 0.0;
        if (live) {
            s = find_slot(nact, q, [&](int k) { return sl[k].row_off; });
            const SlotDesc &d = sl[s];
            const int64_t i = q - d.row_off;
            const uint8_t *rec;
            int nnz;
            locate(d.rows, (uint32_t)i, rec, nnz);
            const int nunits = (nnz + T::U - 1) / T::U;
            double acc = 0.0;
            for (int uu = gl; uu < nunits; uu += G) {
                Unit<ASYRK_F32> un;
                un.load(rec + T::HB + (int64_t)uu * T::UB);
#pragma unroll
                for (int e = 0; e < T::U; ++e)
                    if (uu * T::U + e < nnz) acc = fma((double)un.v[e], d.x64[un.c[e]], acc);
            }
            acc = group_sum<G>(acc);
            const double r = d.b64[i] - acc;
            if (gl == 0) {
                d.side[i].x = r;
                r2 = r * r;
            }
        }
        // one atomic per wave when all its rows belong to one system
        const int s0 = __shfl(s, 0);
        const bool same = __all(!live || s == s0);
        if (same) {
            double w = r2;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off);
            if ((threadIdx.x & 63) == 0 && s0 >= 0) unsafeAtomicAdd(norm2 + s0, w);
        } else if (live && gl == 0) {
            unsafeAtomicAdd(norm2 + s, r2);
        }
    }
}

// ----------------------------------------------------------------- arena

struct Arena {
    uint8_t *base = nullptr;
    int64_t size = 0, used = 0;
    std::map<int64_t, int64_t> free_;  // offset -> length

    static int64_t round_up(int64_t b) { return (b + 255) / 256 * 256; }
    int64_t alloc(int64_t bytes) {
        bytes = round_up(std::max<int64_t>(bytes, 256));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used += bytes;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = round_up(std::max<int64_t>(bytes, 256));
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Request {
    int64_t id = 0;
    int64_t m = 0, n = 0, nnz = 0;
    double tol = 1e-8, b_norm2 = 0.0, fro2 = 0.0, lam = 0.0;
    uint64_t seed = 0;
    SetupResult pack;
    std::vector<double> b64;   // b and the side records {b_i, 1/||a_i||^2} when no
    std::vector<double> side;  // pinned staging block was free at submit
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
    // active state
    int slot = -1;
    int64_t R = 1;
    int64_t off_rec = -1, off_loc = -1, off_b = -1, off_side = -1, off_x = -1, off_d = -1;
    int64_t bytes = 0;
    int64_t rec_bytes = 0;    // packed record bytes
    int64_t dstride = 8;      // bytes per element of the correction d
    int64_t pin_off = -1;     // staging block rec | loc | b64 | side in the pinned arena, or -1
    int64_t pin_bytes = 0;
    int64_t ticket = 0;
    int32_t rounds = 0;
    int32_t next_sweeps = 0;  // sweeps of the request's next round
    int64_t sweeps = 0;
    double rel = 1.0;
    int32_t status = ASYRK_OK;
    std::vector<double> x;  // result
};

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// One of the two groups of active systems.  Their rounds alternate on two
// streams: while the host collects one group's round (retire, admit, slot
// table), the other group's round keeps the GPU busy.
struct RoundGroup {
    hipStream_t st = nullptr;
    TableHead *d_head = nullptr;
    SlotDesc *d_slots = nullptr;
    double *d_norm2 = nullptr;
    TableHead *h_head = nullptr;   // pinned
    SlotDesc *h_slots = nullptr;   // pinned
    double *h_norm2 = nullptr;     // pinned
    hipGraphExec_t graph[2][4] = {};  // per loop (plain / pipelined) and candidate lane width
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEvent_t te[8] = {};         // start / end of each candidate's sweep (lane tuning)
    std::vector<std::unique_ptr<Request>> active;
    // the round in flight (launched, not yet collected)
    bool in_flight = false;
    int pipe = 0, bucket = 0, G = 0;
    bool tune = false;
    int order[4] = {0, 0, 0, 0};
    int64_t workers = 0;
};

}  // namespace

struct asyrk_server {
    asyrk_server_config cfg{};
    Arena arena;
    Arena pinned;                  // host staging arena (pinned), guarded by mu
    RoundGroup grp[2];
    int next_group = 0;            // the group the next progress() call serves
    hipEvent_t e_ref = nullptr;    // time origin of the busy-time union
    double busy_until_ms = 0.0;
    int lanes_last[2] = {4, 16};   // lanes per row of the last plain / pipelined round
    bool tuned_last[2] = {true, true};  // that round ran with a tuned (or fixed) width
    // online choice of the lane width (config lanes / pipe_lanes = 0), per
    // loop and per load bucket (active workers): the bucket's first rounds
    // time every candidate on the same systems
    bool tune_on[2] = {false, false};
    int tuned_G[2][kBuckets] = {};   // 0 while the bucket is being tuned
    int tune_done[2][kBuckets] = {};
    double tune_ms[2][kBuckets][4] = {};
    hipStream_t cst = nullptr;     // admission uploads
    struct Upload {
        hipEvent_t ev;             // recorded on cst after the batch's copies
        std::vector<std::unique_ptr<Request>> reqs;
    };
    std::deque<Upload> uploading;  // admitted batches whose copies may still run
    std::vector<hipEvent_t> ev_pool;
    std::deque<std::unique_ptr<Request>> ready;  // uploaded, waiting for room in a group

    std::mutex mu;
    std::condition_variable cv_submit;  // signalled by submit for an idle run loop
    std::condition_variable cv_pinned;  // signalled when pinned staging is released (or on a fault)
    std::deque<std::unique_ptr<Request>> queue;
    std::unordered_map<int64_t, std::unique_ptr<Request>> done;
    std::unordered_set<int64_t> live;  // submitted and not yet polled
    std::vector<int64_t> finished;     // completed ids not yet reported by take_completed
    int64_t next_id = 1;

    std::atomic<int64_t> n_active{0};  // admitted and not finished, for other threads
    int64_t workers_in_use = 0;        // R over admitted requests not yet finished
    asyrk_server_stats stats{};
    // the first device failure of a round: sticky, every later progress,
    // submit and poll of an unfinished request returns it
    std::atomic<int> fault{ASYRK_OK};
};

namespace {

thread_local const char *g_srv_last = "";

asyrk_status srv_fail(hipError_t e) {
    g_srv_last = hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? ASYRK_ERR_OOM : ASYRK_ERR_DEVICE;
}

#define SRV_OK(expr)                                  \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return srv_fail(_e);    \
    } while (0)

int64_t request_bytes(const Request &r) {
    return Arena::round_up(r.rec_bytes) + Arena::round_up((int64_t)r.pack.loc.size() * 8) +
           Arena::round_up(r.m * 8) + Arena::round_up(r.m * 16) + Arena::round_up(r.n * 8) +
           Arena::round_up(r.n * r.dstride) + 6 * 256;
}

constexpr int kTunePasses = 2;  // tuning rounds per candidate (each candidate runs first once per pass)

// Load bucket of a round for lane tuning: powers of two of the active
// workers, from pipe_workers / 8 (pipelined rounds) or pipe_workers (plain).
int load_bucket(int64_t workers, int64_t base) {
    int b = 0;
    for (int64_t lim = std::max<int64_t>(1, base) * 2; b < kBuckets - 1 && workers >= lim; lim *= 2) ++b;
    return b;
}

int cand_index(int pipe, int G) {
    for (int k = 0; k < kNumCands[pipe]; ++k)
        if (kLaneCands[pipe][k] == G) return k;
    return 0;
}

// zero d and the norms, then one sweep over every active system of a group
// with G lanes per row; the grid covers max_workers workers (pipelined:
// pipe_workers)
hipError_t launch_zero_and_sweep(const asyrk_server *s, const RoundGroup &g, hipStream_t st, int pipe, int G) {
    hipLaunchKernelGGL(srv_zero_kernel, dim3(kVecBlocks), dim3(256), 0, st, g.d_head, g.d_slots, g.d_norm2);
    const int64_t workers = pipe ? std::min<int64_t>(s->cfg.max_workers, s->cfg.pipe_workers) : s->cfg.max_workers;
    const int block = pipe ? 64 : 256;  // light rounds: one wave per block, spread over the CUs
    const dim3 grid((unsigned)((workers * G + block - 1) / block));
    if (pipe && s->cfg.order == 1) {
        switch (G) {
            case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(srv_sweep_pipe_kernel<4, true>), grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(srv_sweep_pipe_kernel<8, true>), grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            case 16: hipLaunchKernelGGL(HIP_KERNEL_NAME(srv_sweep_pipe_kernel<16, true>), grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            case 32: hipLaunchKernelGGL(HIP_KERNEL_NAME(srv_sweep_pipe_kernel<32, true>), grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            default: return hipErrorInvalidValue;
        }
    } else if (pipe) {
        switch (G) {
            case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(srv_sweep_pipe_kernel<4, false>), grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            case 8: hipLaunchKernelGGL(HIP_KERNEL_NAME(srv_sweep_pipe_kernel<8, false>), grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            case 16: hipLaunchKernelGGL(HIP_KERNEL_NAME(srv_sweep_pipe_kernel<16, false>), grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            case 32: hipLaunchKernelGGL(HIP_KERNEL_NAME(srv_sweep_pipe_kernel<32, false>), grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            default: return hipErrorInvalidValue;
        }
    } else if (s->cfg.order == 1) {
        switch (G) {
            case 4: hipLaunchKernelGGL(srv_sweep_slices_kernel<4>, grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            case 8: hipLaunchKernelGGL(srv_sweep_slices_kernel<8>, grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (G) {
            case 4: hipLaunchKernelGGL(srv_sweep_kernel<4>, grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            case 8: hipLaunchKernelGGL(srv_sweep_kernel<8>, grid, dim3(block), 0, st, g.d_head, g.d_slots); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_finish(const RoundGroup &g, hipStream_t st) {
    hipLaunchKernelGGL(srv_axpy_kernel, dim3(kVecBlocks), dim3(256), 0, st, g.d_head, g.d_slots);
    hipLaunchKernelGGL(srv_residual_kernel, dim3(kVecBlocks), dim3(256), 0, st, g.d_head, g.d_slots, g.d_norm2);
    return hipGetLastError();
}

hipError_t launch_round(const asyrk_server *s, const RoundGroup &g, hipStream_t st, int pipe, int G) {
    hipError_t e = launch_zero_and_sweep(s, g, st, pipe, G);
    return e == hipSuccess ? launch_finish(g, st) : e;
}

// Capture a group's round of one sweep variant and lane width as a graph;
// the kernels read the group's slot table, so one graph serves every round
// whatever systems are active.
hipError_t capture_round(const asyrk_server *s, RoundGroup &g, int pipe, int k) {
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamBeginCapture(g.st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = launch_round(s, g, g.st, pipe, kLaneCands[pipe][k]);
        e = hipStreamEndCapture(g.st, &gr);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g.graph[pipe][k], gr, nullptr, nullptr, 0);
    if (gr) (void)hipGraphDestroy(gr);
    return e;
}

void free_server(asyrk_server *s) {
    if (!s) return;
    for (RoundGroup &g : s->grp)
        if (g.st) (void)hipStreamSynchronize(g.st);
    if (s->cst) (void)hipStreamSynchronize(s->cst);
    for (RoundGroup &g : s->grp) {
        for (auto &row : g.graph)
            for (hipGraphExec_t x : row)
                if (x) (void)hipGraphExecDestroy(x);
        (void)hipFree(g.d_head);
        (void)hipFree(g.d_slots);
        (void)hipFree(g.d_norm2);
        if (g.h_head) (void)hipHostFree(g.h_head);
        if (g.h_slots) (void)hipHostFree(g.h_slots);
        if (g.h_norm2) (void)hipHostFree(g.h_norm2);
        if (g.e0) (void)hipEventDestroy(g.e0);
        if (g.e1) (void)hipEventDestroy(g.e1);
        for (hipEvent_t ev : g.te)
            if (ev) (void)hipEventDestroy(ev);
        if (g.st) (void)hipStreamDestroy(g.st);
    }
    (void)hipFree(s->arena.base);
    if (s->pinned.base) (void)hipHostFree(s->pinned.base);
    if (s->e_ref) (void)hipEventDestroy(s->e_ref);
    if (s->cst) (void)hipStreamDestroy(s->cst);
    for (auto &u : s->uploading)
        if (u.ev) (void)hipEventDestroy(u.ev);
    for (hipEvent_t ev : s->ev_pool) (void)hipEventDestroy(ev);
    delete s;
}

}  // namespace

extern "C" {

void asyrk_server_config_init(asyrk_server_config *c) {
    if (!c) return;
    std::memset(c, 0, sizeof *c);
    c->budget_bytes = (int64_t)64 << 30;
    c->max_slots = 1024;
    c->max_workers = (int64_t)1 << 16;
    c->inner_sweeps = 8;
    c->max_rounds = 60;
    c->gamma = 1.0;
    c->use_graph = 1;
    c->pinned_bytes = (int64_t)4 << 30;
    c->lanes = 4;
    c->pipe_workers = 8192;
    c->pipe_lanes = 16;
    c->order = 1;
    c->pinned_wait_ms = 1000;
}

asyrk_status asyrk_server_create(asyrk_server **out, const asyrk_server_config *cfg_in) {
    if (!out) return ASYRK_ERR_INVALID_ARG;
    *out = nullptr;
    asyrk_server_config cfg;
    if (cfg_in)
        cfg = *cfg_in;
    else
        asyrk_server_config_init(&cfg);
    if (cfg.budget_bytes < (1 << 20) || cfg.pinned_bytes < 0 || cfg.max_slots < 1 || cfg.max_slots > 65536 || cfg.max_workers < 64 ||
        cfg.max_workers > ((int64_t)1 << 24) || cfg.inner_sweeps < 1 || cfg.max_rounds < 1 ||
        !(cfg.gamma > 0.0 && cfg.gamma < 2.0) || (cfg.lanes != 0 && cfg.lanes != 4 && cfg.lanes != 8) ||
        cfg.pipe_workers < 0 || (cfg.pipe_lanes != 0 && cfg.pipe_lanes != 4 && cfg.pipe_lanes != 8 && cfg.pipe_lanes != 16 &&
                                  cfg.pipe_lanes != 32) ||
        (cfg.fixed_rounds != 0 && cfg.fixed_rounds != 1) || (cfg.order != 0 && cfg.order != 1) ||
        cfg.pinned_wait_ms < 0)
        return ASYRK_ERR_INVALID_ARG;
    asyrk_server *s = new (std::nothrow) asyrk_server();
    if (!s) return ASYRK_ERR_OOM;
    s->cfg = cfg;
    s->lanes_last[0] = cfg.lanes ? cfg.lanes : 4;
    s->lanes_last[1] = cfg.pipe_lanes ? cfg.pipe_lanes : 16;
    s->tune_on[0] = cfg.lanes == 0;
    s->tune_on[1] = cfg.pipe_lanes == 0 && cfg.pipe_workers > 0;
    for (int pipe = 0; pipe < 2; ++pipe)
        for (int b = 0; b < kBuckets; ++b) s->tuned_G[pipe][b] = s->tune_on[pipe] ? 0 : s->lanes_last[pipe];
    hipError_t e = hipMalloc((void **)&s->arena.base, (size_t)cfg.budget_bytes);
    for (RoundGroup &g : s->grp) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&g.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMalloc((void **)&g.d_head, sizeof(TableHead));
        if (e == hipSuccess) e = hipMalloc((void **)&g.d_slots, sizeof(SlotDesc) * cfg.max_slots);
        if (e == hipSuccess) e = hipMalloc((void **)&g.d_norm2, sizeof(double) * cfg.max_slots);
        if (e == hipSuccess) e = hipHostMalloc((void **)&g.h_head, sizeof(TableHead), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&g.h_slots, sizeof(SlotDesc) * cfg.max_slots, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&g.h_norm2, sizeof(double) * cfg.max_slots, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreate(&g.e0);
        if (e == hipSuccess) e = hipEventCreate(&g.e1);
        for (int k = 0; k < 8 && e == hipSuccess && (s->tune_on[0] || s->tune_on[1]); ++k) e = hipEventCreate(&g.te[k]);
        if (e == hipSuccess) std::memset(g.h_head, 0, sizeof(TableHead));
    }
    if (e == hipSuccess && cfg.pinned_bytes > 0)
        e = hipHostMalloc((void **)&s->pinned.base, (size_t)cfg.pinned_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->cst, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&s->e_ref);
    if (e == hipSuccess) e = hipEventRecord(s->e_ref, s->grp[0].st);
    if (e == hipSuccess && cfg.use_graph) {
        // the four phases captured per group, sweep variant and lane width in use
        for (RoundGroup &g : s->grp)
            for (int pipe = 0; pipe < 2 && e == hipSuccess; ++pipe) {
                if (pipe && cfg.pipe_workers == 0) break;
                for (int k = 0; k < kNumCands[pipe] && e == hipSuccess; ++k)
                    if (s->tune_on[pipe] || kLaneCands[pipe][k] == s->lanes_last[pipe]) e = capture_round(s, g, pipe, k);
            }
    }
    if (e != hipSuccess) {
        free_server(s);
        return srv_fail(e);
    }
    s->arena.size = cfg.budget_bytes;
    s->arena.free_[0] = cfg.budget_bytes;
    if (cfg.pinned_bytes > 0) {
        s->pinned.size = cfg.pinned_bytes;
        s->pinned.free_[0] = cfg.pinned_bytes;
    }
    *out = s;
    return ASYRK_OK;
}

asyrk_status asyrk_server_destroy(asyrk_server *s) {
    free_server(s);
    return ASYRK_OK;
}

asyrk_status asyrk_server_submit(asyrk_server *s, int64_t m, int64_t n, const int64_t *row_ptr,
                                 const int32_t *col_idx, const float *vals, const double *b, double tol,
                                 uint64_t seed, int64_t *request_id) {
    if (!s || !request_id || !(tol > 0.0) || !std::isfinite(tol)) return ASYRK_ERR_INVALID_ARG;
    if (s->fault.load() != ASYRK_OK) return (asyrk_status)s->fault.load();
    auto r = std::unique_ptr<Request>(new (std::nothrow) Request());
    if (!r) return ASYRK_ERR_OOM;
    asyrk_status rc = validate_system(m, n, row_ptr, col_idx, vals, ASYRK_F32, b, r->pack);
    if (rc) return rc;
    std::vector<uint32_t> thresh;
    std::vector<int32_t> alias;
    build_alias(r->pack.w, thresh, alias);
    rc = plan_records(m, row_ptr, ASYRK_F32, r->pack, &r->rec_bytes);
    if (rc) return rc;
    r->m = m;
    r->n = n;
    r->nnz = r->pack.nnz;
    r->tol = tol;
    r->seed = seed;
    double bn = 0.0;
    for (int64_t i = 0; i < m; ++i) bn += b[i] * b[i];
    r->b_norm2 = bn;
    r->fro2 = r->pack.fro2;
    const double q = std::sqrt((double)n / (double)m);
    r->lam = std::max((1.0 + q) * (1.0 + q) * r->fro2 / (double)n, r->pack.max_col_norm2);
    r->dstride = iterate_stride(n);
    r->bytes = request_bytes(*r);
    if (r->bytes > s->cfg.budget_bytes) return ASYRK_ERR_OOM;
    // The records, locators, b and the first round's side records
    // {r_0 = b (x_0 = 0), 1/||a_i||^2} are written straight into a pinned
    // staging block laid out as rec | loc | b64 | side, so admission is one
    // DMA; without room there they go to pageable vectors.
    const int64_t lrec = Arena::round_up(r->rec_bytes);
    const int64_t lloc = Arena::round_up((int64_t)r->pack.loc.size() * 8);
    const int64_t lb = Arena::round_up(m * 8);
    const int64_t lside = Arena::round_up(m * 16);
    // Pinned staging full: wait (up to pinned_wait_ms) for uploads to release
    // some, so that admissions stay DMA transfers; a pageable request's upload
    // would hold the round loop's thread for its whole copy exactly when the
    // queue is longest.
    int64_t off = -1;
    if (s->pinned.base) {
        const int64_t need = lrec + lloc + lb + lside;
        std::unique_lock<std::mutex> lk(s->mu);
        off = s->pinned.alloc(need);
        if (off < 0 && need <= s->pinned.size && s->cfg.pinned_wait_ms > 0) {
            const auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(s->cfg.pinned_wait_ms);
            while (off < 0 && s->fault.load() == ASYRK_OK &&
                   s->cv_pinned.wait_until(lk, until) != std::cv_status::timeout)
                off = s->pinned.alloc(need);
            if (off < 0) off = s->pinned.alloc(need);
        }
    }
    uint8_t *p_rec, *p_b, *p_side;
    if (off >= 0) {
        uint8_t *p = s->pinned.base + off;
        p_rec = p;
        if (!r->pack.loc.empty()) std::memcpy(p + lrec, r->pack.loc.data(), r->pack.loc.size() * 8);
        p_b = p + lrec + lloc;
        p_side = p + lrec + lloc + lb;
        r->pin_off = off;
        r->pin_bytes = lrec + lloc + lb + lside;
    } else {
        try {
            r->pack.rec.resize((size_t)r->rec_bytes);
            r->b64.resize((size_t)m);
            r->side.resize((size_t)m * 2);
        } catch (...) {
            return ASYRK_ERR_OOM;
        }
        p_rec = r->pack.rec.data();
        p_b = reinterpret_cast<uint8_t *>(r->b64.data());
        p_side = reinterpret_cast<uint8_t *>(r->side.data());
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.pageable_uploads++;
    }
    write_records(m, row_ptr, col_idx, vals, ASYRK_F32, b, r->pack, thresh.data(), alias.data(), p_rec);
    std::memcpy(p_b, b, (size_t)m * 8);
    double *side = reinterpret_cast<double *>(p_side);
    for (int64_t i = 0; i < m; ++i) {
        side[2 * i] = b[i];
        side[2 * i + 1] = 1.0 / r->pack.w[i];
    }
    r->t_submit = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    *request_id = r->id;
    s->live.insert(r->id);
    s->queue.push_back(std::move(r));
    s->stats.submitted++;
    s->cv_submit.notify_one();
    return ASYRK_OK;
}

}  // extern "C"

namespace {

// Wait for a group's round, account for it, size the next round of every
// request that goes on, and retire the ones that finished.
asyrk_status collect_round(asyrk_server *s, RoundGroup &g) {
    const asyrk_server_config &cfg = s->cfg;
    SRV_OK(hipStreamSynchronize(g.st));
    g.in_flight = false;
    float ms = 0.f, t0 = 0.f, t1 = 0.f;
    SRV_OK(hipEventElapsedTime(&ms, g.e0, g.e1));
    SRV_OK(hipEventElapsedTime(&t0, s->e_ref, g.e0));
    SRV_OK(hipEventElapsedTime(&t1, s->e_ref, g.e1));
    const int pipe = g.pipe, bucket = g.bucket, nc = kNumCands[pipe];
    if (g.tune) {
        for (int k = 0; k < nc; ++k) {
            float t = 0.f;
            SRV_OK(hipEventElapsedTime(&t, g.te[2 * k], g.te[2 * k + 1]));
            s->tune_ms[pipe][bucket][g.order[k]] += t;
        }
        if (++s->tune_done[pipe][bucket] == kTunePasses * nc) {
            int best = 0;
            for (int k = 1; k < nc; ++k)
                if (s->tune_ms[pipe][bucket][k] < s->tune_ms[pipe][bucket][best]) best = k;
            std::lock_guard<std::mutex> lk(s->mu);
            s->tuned_G[pipe][bucket] = kLaneCands[pipe][best];
        }
    }
    const int nact = (int)g.active.size();
    int64_t round_rows = 0;
    for (const auto &r : g.active) round_rows += (int64_t)r->next_sweeps * r->m;
    {
        std::lock_guard<std::mutex> lk(s->mu);  // stats are read by other threads
        // busy time: the union of the rounds' intervals on the two streams
        const double a = std::max<double>(t0, s->busy_until_ms);
        if (t1 > a) s->stats.gpu_seconds += (t1 - a) * 1e-3;
        s->busy_until_ms = std::max<double>(s->busy_until_ms, t1);
        s->stats.rounds++;
        s->stats.row_updates += round_rows;
        s->stats.round_workers += g.workers;
        s->stats.round_systems += nact;
        s->stats.pipelined_rounds += pipe;
        s->lanes_last[pipe] = g.G;
        s->tuned_last[pipe] = !g.tune;
    }
    (void)ms;
    // ---- bookkeeping and retirement: every finished x is copied out, then one wait
    // (every device call comes before any request leaves g.active, so a
    // failure leaves the group as it was)
    uint8_t *base = s->arena.base;
    std::vector<char> retire((size_t)nact, 0);
    for (int k = 0; k < nact; ++k) {
        std::unique_ptr<Request> &r = g.active[k];
        const int ns = r->next_sweeps;
        r->ticket += (int64_t)ns * r->m;
        r->sweeps += ns;
        r->rounds++;
        const double nr = g.h_norm2[k];
        const double prev = r->rel;
        r->rel = r->b_norm2 > 0 ? std::sqrt(nr / r->b_norm2) : std::sqrt(nr);
        const bool conv = r->rel <= r->tol;
        const bool bad = !std::isfinite(r->rel);
        if (conv || bad || r->rounds >= cfg.max_rounds) {
            r->status = conv ? ASYRK_OK : (bad ? ASYRK_ERR_DIVERGED : ASYRK_ERR_NOT_CONVERGED);
            r->x.resize(r->n);
            SRV_OK(hipMemcpyAsync(r->x.data(), base + r->off_x, r->n * 8, hipMemcpyDeviceToHost, g.st));
            retire[k] = 1;
        } else {
            // Size the next round from this one: RK contracts the residual by
            // a roughly constant factor per sweep, so the sweeps still needed
            // are log(tol / rel) / log(rho), rho the factor measured over the
            // round just run; one more for safety, at most inner_sweeps.
            int nxt = cfg.inner_sweeps;
            if (!cfg.fixed_rounds && prev > 0.0 && r->rel > 0.0 && r->rel < prev) {
                const double rho = std::pow(r->rel / prev, 1.0 / ns);
                const double need = std::log(r->tol / r->rel) / std::log(rho);
                if (std::isfinite(need))
                    nxt = (int)std::min<double>(cfg.inner_sweeps, std::max(1.0, std::ceil(need) + 1.0));
            }
            r->next_sweeps = nxt;
        }
    }
    bool any_out = false;
    for (int k = 0; k < nact; ++k) any_out |= retire[k] != 0;
    if (any_out) SRV_OK(hipStreamSynchronize(g.st));
    std::vector<std::unique_ptr<Request>> keep, out;
    for (int k = 0; k < nact; ++k) (retire[k] ? out : keep).push_back(std::move(g.active[k]));
    g.active.swap(keep);
    if (!out.empty()) {
        const double t = now_s();
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &r : out) {
            r->t_done = t;
            s->workers_in_use -= r->R;
            s->arena.release(r->off_rec, r->bytes);
            r->pack = SetupResult();  // drop the packed copy
            s->stats.completed++;
            s->finished.push_back(r->id);
            s->done[r->id] = std::move(r);
        }
    }
    return ASYRK_OK;
}

}  // namespace

extern "C" {

static asyrk_status server_progress(asyrk_server *s, int32_t *n_active, int32_t *n_queued);

asyrk_status asyrk_server_progress(asyrk_server *s, int32_t *n_active, int32_t *n_queued) {
    if (!s) return ASYRK_ERR_INVALID_ARG;
    const int f = s->fault.load();
    if (f != ASYRK_OK) return (asyrk_status)f;
    const asyrk_status rc = server_progress(s, n_active, n_queued);
    if (rc != ASYRK_OK) {
        s->fault.store(rc);
        s->cv_pinned.notify_all();  // submits waiting for staging give up
    }
    return rc;
}

static asyrk_status server_progress(asyrk_server *s, int32_t *n_active, int32_t *n_queued) {
    const asyrk_server_config &cfg = s->cfg;
    // The two groups take turns: collect this group's previous round while
    // the other group's round computes, admit into this group, launch its
    // next round.
    RoundGroup &g = s->grp[s->next_group];
    RoundGroup &other = s->grp[s->next_group ^ 1];
    s->next_group ^= 1;
    if (g.in_flight) {
        asyrk_status rc = collect_round(s, g);
        if (rc) return rc;
    }
    // ---- uploads that have finished make their requests ready; when the GPU
    // would otherwise have nothing to do, wait for the oldest batch
    using Upload = asyrk_server::Upload;
    auto finish_upload = [&](Upload &u) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (auto &r : u.reqs) {
                if (r->pin_off >= 0) {
                    s->pinned.release(r->pin_off, r->pin_bytes);
                    r->pin_off = -1;
                }
                s->ready.push_back(std::move(r));
            }
            s->ev_pool.push_back(u.ev);
        }
        s->cv_pinned.notify_all();
    };
    while (!s->uploading.empty()) {
        Upload &u = s->uploading.front();
        const hipError_t q = hipEventQuery(u.ev);
        if (q == hipErrorNotReady) {
            if (!g.active.empty() || other.in_flight || !s->ready.empty()) break;
            SRV_OK(hipEventSynchronize(u.ev));
        } else if (q != hipSuccess) {
            return srv_fail(q);
        }
        finish_upload(u);
        s->uploading.pop_front();
    }
    // ---- ready requests join this group: a round's worker grid covers
    // max_workers, and both groups together hold at most one and a half times
    // that
    int64_t g_workers = 0, o_workers = 0;
    for (const auto &r : g.active) g_workers += r->R;
    for (const auto &r : other.active) o_workers += r->R;
    const int64_t total_cap = cfg.max_workers + cfg.max_workers / 2;
    while (!s->ready.empty() && (int64_t)g.active.size() < cfg.max_slots) {
        const int64_t R = s->ready.front()->R;
        if (g_workers + R > cfg.max_workers || g_workers + o_workers + R > total_cap) break;
        g_workers += R;
        g.active.push_back(std::move(s->ready.front()));
        s->ready.pop_front();
    }
    // ---- admit: uploads on the copy stream, for a later call to pick up; the
    // admitted requests may hold up to half of max_workers beyond the two
    // groups' active workers, so that uploads run ahead of the rounds
    Upload batch{};
    for (;;) {
        std::unique_ptr<Request> r;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->queue.empty()) break;
            Request &f = *s->queue.front();
            int64_t R = (int64_t)std::floor(f.fro2 / (2.0 * M_E * f.lam));
            R = std::max<int64_t>(1, std::min<int64_t>(R, cfg.max_workers / 4));
            if (s->workers_in_use + R > 2 * cfg.max_workers) break;
            f.R = R;
            const int64_t off = s->arena.alloc(f.bytes);
            if (off < 0) break;  // wait for memory
            r = std::move(s->queue.front());
            s->queue.pop_front();
            r->off_rec = off;
        }
        Request &q = *r;
        int64_t o = q.off_rec + Arena::round_up(q.rec_bytes);
        q.off_loc = o;
        o += Arena::round_up((int64_t)q.pack.loc.size() * 8);
        q.off_b = o;
        o += Arena::round_up(q.m * 8);
        q.off_side = o;
        o += Arena::round_up(q.m * 16);
        q.off_x = o;
        o += Arena::round_up(q.n * 8);
        q.off_d = o;
        uint8_t *base = s->arena.base;
        if (q.pin_off >= 0) {
            // one DMA of the staged rec | loc | b64 | side block (same relative layout)
            SRV_OK(hipMemcpyAsync(base + q.off_rec, s->pinned.base + q.pin_off, q.pin_bytes, hipMemcpyHostToDevice,
                                  s->cst));
        } else {
            SRV_OK(hipMemcpyAsync(base + q.off_rec, q.pack.rec.data(), q.rec_bytes, hipMemcpyHostToDevice,
                                  s->cst));
            if (!q.pack.loc.empty())
                SRV_OK(hipMemcpyAsync(base + q.off_loc, q.pack.loc.data(), q.pack.loc.size() * 8,
                                      hipMemcpyHostToDevice, s->cst));
            SRV_OK(hipMemcpyAsync(base + q.off_b, q.b64.data(), q.m * 8, hipMemcpyHostToDevice, s->cst));
            SRV_OK(hipMemcpyAsync(base + q.off_side, q.side.data(), q.m * 16, hipMemcpyHostToDevice, s->cst));
        }
        SRV_OK(launch_zero(base + q.off_x, q.n * 8, s->cst));
        q.t_admit = now_s();
        q.rel = q.b_norm2 > 0 ? 1.0 : 0.0;
        q.next_sweeps = cfg.inner_sweeps;
        batch.reqs.push_back(std::move(r));
        std::lock_guard<std::mutex> lk(s->mu);  // stats are read by other threads
        s->workers_in_use += q.R;
        s->stats.admitted++;
    }
    if (!batch.reqs.empty()) {
        if (s->ev_pool.empty()) {
            hipEvent_t ev = nullptr;
            SRV_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            s->ev_pool.push_back(ev);
        }
        batch.ev = s->ev_pool.back();
        s->ev_pool.pop_back();
        SRV_OK(hipEventRecord(batch.ev, s->cst));
        s->uploading.push_back(std::move(batch));
        if (g.active.empty() && !other.in_flight) {
            // nothing else for the GPU: this group's round takes the batch now
            Upload &u = s->uploading.back();
            SRV_OK(hipEventSynchronize(u.ev));
            // (older batches finished before it on the same stream)
            while (!s->uploading.empty()) {
                finish_upload(s->uploading.front());
                s->uploading.pop_front();
            }
            while (!s->ready.empty() && (int64_t)g.active.size() < cfg.max_slots) {
                const int64_t R = s->ready.front()->R;
                if (g_workers + R > cfg.max_workers || g_workers + o_workers + R > total_cap) break;
                g_workers += R;
                g.active.push_back(std::move(s->ready.front()));
                s->ready.pop_front();
            }
        }
    }
    if (!g.active.empty()) {
        // ---- slot table
        TableHead &h = *g.h_head;
        h.nact = (int32_t)g.active.size();
        int64_t wo = 0, ro = 0, co = 0;
        uint8_t *base = s->arena.base;
        for (int k = 0; k < h.nact; ++k) {
            Request &q = *g.active[k];
            SlotDesc &d = g.h_slots[k];
            d.rows.rec = base + q.off_rec;
            d.rows.loc = q.pack.loc.empty() ? nullptr : reinterpret_cast<const RowLoc *>(base + q.off_loc);
            d.rows.stride = q.pack.stride;
            d.rows.fixed_nnz = (int32_t)q.pack.fixed_nnz;
            d.rows.m = (int32_t)q.m;
            d.b64 = reinterpret_cast<double *>(base + q.off_b);
            d.x64 = reinterpret_cast<double *>(base + q.off_x);
            d.d = reinterpret_cast<double *>(base + q.off_d);
            d.side = reinterpret_cast<double2 *>(base + q.off_side);
            d.n = q.n;
            d.R = q.R;
            d.w_off = wo;
            d.row_off = ro;
            d.col_off = co;
            d.t_begin = q.ticket;
            d.t_end = q.ticket + (int64_t)q.next_sweeps * q.m;
            d.key0 = (uint32_t)q.seed;
            d.key1 = (uint32_t)(q.seed >> 32);
            d.gamma = cfg.gamma;
            d.xshift = stride_shift(q.dstride, 8);
            d.pad = 0;
            wo += q.R;
            ro += q.m;
            co += q.n;
        }
        // the captured grids cover max_workers workers (pipelined: pipe_workers)
        if (wo > cfg.max_workers) {
            g_srv_last = "internal: active workers exceed max_workers";
            return ASYRK_ERR_DEVICE;
        }
        h.total_workers = wo;
        h.total_rows = ro;
        h.total_cols = co;
        SRV_OK(hipMemcpyAsync(g.d_head, g.h_head, sizeof(TableHead), hipMemcpyHostToDevice, g.st));
        SRV_OK(hipMemcpyAsync(g.d_slots, g.h_slots, sizeof(SlotDesc) * h.nact, hipMemcpyHostToDevice, g.st));
        // ---- launch the round
        g.pipe = h.total_workers <= cfg.pipe_workers ? 1 : 0;
        g.bucket = g.pipe ? load_bucket(h.total_workers, cfg.pipe_workers / 8) : load_bucket(h.total_workers, cfg.pipe_workers);
        g.tune = s->tuned_G[g.pipe][g.bucket] == 0;
        g.workers = wo;
        const int nc = kNumCands[g.pipe];
        SRV_OK(hipEventRecord(g.e0, g.st));
        if (g.tune) {
            // every candidate sweeps this round's systems from d = 0, timed; the
            // last one's sweep is the round's (the order rotates so that each
            // candidate also runs first, on cold caches)
            for (int k = 0; k < nc; ++k) g.order[k] = (s->tune_done[g.pipe][g.bucket] + k) % nc;
            for (int k = 0; k < nc; ++k) {
                SRV_OK(hipEventRecord(g.te[2 * k], g.st));
                SRV_OK(launch_zero_and_sweep(s, g, g.st, g.pipe, kLaneCands[g.pipe][g.order[k]]));
                SRV_OK(hipEventRecord(g.te[2 * k + 1], g.st));
            }
            SRV_OK(launch_finish(g, g.st));
            g.G = kLaneCands[g.pipe][g.order[nc - 1]];
        } else {
            g.G = s->tuned_G[g.pipe][g.bucket];
            hipGraphExec_t gx = g.graph[g.pipe][cand_index(g.pipe, g.G)];
            if (gx)
                SRV_OK(hipGraphLaunch(gx, g.st));
            else
                SRV_OK(launch_round(s, g, g.st, g.pipe, g.G));
        }
        SRV_OK(hipEventRecord(g.e1, g.st));
        SRV_OK(hipMemcpyAsync(g.h_norm2, g.d_norm2, sizeof(double) * h.nact, hipMemcpyDeviceToHost, g.st));
        g.in_flight = true;
    }
    int64_t act = (int64_t)(s->grp[0].active.size() + s->grp[1].active.size() + s->ready.size());
    for (const auto &u : s->uploading) act += (int64_t)u.reqs.size();
    s->n_active.store(act);
    if (n_active) *n_active = (int32_t)act;
    if (n_queued) {
        std::lock_guard<std::mutex> lk(s->mu);
        *n_queued = (int32_t)s->queue.size();
    }
    return ASYRK_OK;
}

asyrk_status asyrk_server_run(asyrk_server *s, const volatile int32_t *stop) {
    if (!s || !stop) return ASYRK_ERR_INVALID_ARG;
    while (*stop == 0) {
        int32_t act = 0, q = 0;
        const asyrk_status rc = asyrk_server_progress(s, &act, &q);
        if (rc) return rc;
        if (act == 0 && q == 0) {
            // idle: sleep until a submit (or 1 ms, to see the stop flag)
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->queue.empty()) s->cv_submit.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
    return ASYRK_OK;
}

asyrk_status asyrk_server_poll(asyrk_server *s, int64_t request_id, double *x_out, asyrk_request_stats *st) {
    if (!s) return ASYRK_ERR_INVALID_ARG;
    std::unique_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->done.find(request_id);
        if (it == s->done.end()) {
            if (!s->live.count(request_id)) return ASYRK_ERR_INVALID_ARG;
            const int f = s->fault.load();
            return f != ASYRK_OK ? (asyrk_status)f : ASYRK_PENDING;
        }
        r = std::move(it->second);
        s->done.erase(it);
        s->live.erase(request_id);
    }
    if (x_out) std::memcpy(x_out, r->x.data(), r->n * 8);
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->m = r->m;
        st->n = r->n;
        st->nnz = r->nnz;
        st->rounds = r->rounds;
        st->in_flight = r->R;
        st->sweeps = r->sweeps;
        st->rel_residual = r->rel;
        st->t_submit = r->t_submit;
        st->t_admit = r->t_admit;
        st->t_done = r->t_done;
        st->status = r->status;
    }
    return (asyrk_status)r->status;
}

asyrk_status asyrk_server_stats_get(asyrk_server *s, asyrk_server_stats *out) {
    if (!s || !out) return ASYRK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->active = s->n_active.load();
    out->queued = (int64_t)s->queue.size();
    out->arena_used = s->arena.used;
    out->lanes = s->lanes_last[0];
    out->pipe_lanes = s->lanes_last[1];
    out->lanes_tuning = (int32_t)!s->tuned_last[0] | ((int32_t)!s->tuned_last[1] << 1);
    int32_t left = 0;
    for (int pipe = 0; pipe < 2; ++pipe)
        for (int b = 0; b < kBuckets; ++b) left += s->tuned_G[pipe][b] == 0;
    out->buckets_untuned = left;
    return ASYRK_OK;
}

asyrk_status asyrk_server_take_completed(asyrk_server *s, int64_t *ids, int64_t cap, int64_t *count) {
    if (!s || !count || cap < 0 || (cap > 0 && !ids)) return ASYRK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t k = std::min<int64_t>(cap, (int64_t)s->finished.size());
    std::copy(s->finished.begin(), s->finished.begin() + k, ids);
    s->finished.erase(s->finished.begin(), s->finished.begin() + k);
    *count = k;
    return ASYRK_OK;
}

double asyrk_now(void) { return now_s(); }

}  // extern "C"
