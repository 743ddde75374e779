// C ABI of the asynchronous randomized Kaczmarz library (include/asyrk.h):
// system creation, the solve driver (async, replay, refinement), residual,
// sampler exposure, lambda_max and device ceilings.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "device.h"
#include "setup.h"
#include "setup_dev.h"

using namespace asyrk;

struct asyrk_system {
    int64_t m = 0, n = 0, nnz = 0;
    int32_t vk = ASYRK_F32;
    int32_t mem = ASYRK_MEM_HOST;
    hipStream_t st = nullptr;
    int64_t mu = 0, nu = 0, fixed_nnz = 0, stride = 0;
    double fro2 = 0.0, max_col_norm2 = 0.0;
    Rows rows{};
    uint8_t *d_rec = nullptr;
    int64_t rec_bytes = 0;        // size of the record image
    RowLoc *d_loc = nullptr;
    double *d_b64 = nullptr;
    void *d_x = nullptr;          // sweep iterate: element c at byte c * xstride (float or double)
    int64_t xstride = 8;          // bytes per iterate element (a power of two >= 8)
    double2 *d_side = nullptr;    // {b_i, 1/w_i} in FP64 for FP64 iterates over FP32/BF16 records
    double *d_x64 = nullptr;      // FP64 master iterate
    double *d_xref = nullptr;     // FP64 reference for the error monitor
    double *d_part = nullptr;     // reduction partials
    double *d_scalar = nullptr;   // 4 device scalars
    double *h_pin = nullptr;      // 4 pinned host scalars
    uint64_t *d_trace = nullptr;  // staleness samples, kTraceWords per wave
    int64_t trace_cap = 0;        // waves d_trace holds
    uint64_t *d_tau = nullptr;    // the completion counter's shards (monotone, never reset)
    double lambda_pi = 0.0;       // lambda_max by power iteration, once asyrk_lambda_max ran (else 0)
    int64_t aug_n = 0;            // augmented system: columns of the original A (else 0)
    double aug_zeta = 0.0;        // augmented system: its zeta
    int64_t device_bytes = 0;
    bool rec_b_dirty = false;
    int tuned_G[2] = {0, 0};      // autotuned lanes per row for F64 / F32 iterates (0 = none)
    int tuned_pipe[2] = {0, 0};   // autotuned worker loop (0 plain, 1 pipelined, 2 batched) for F64 / F32 iterates
    int64_t tuned_R[2] = {0, 0};  // the R those were tuned at
    bool tuned_auto_R[2] = {false, false};  // R chosen by the autotuner: solves with in_flight = 0 use it
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int dev = 0;                  // the device current at creation (its stream's device)
};

namespace {

thread_local const char *g_last = "";


asyrk_status dev_fail(hipError_t e) {
    g_last = hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? ASYRK_ERR_OOM : ASYRK_ERR_DEVICE;
}

#define HIP_OK(expr)                                  \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return dev_fail(_e);    \
    } while (0)

template <class T>
hipError_t dmalloc(asyrk_system *s, T **p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e == hipSuccess) s->device_bytes += (int64_t)bytes;
    return e;
}

void free_system(asyrk_system *s) {
    if (!s) return;
    if (s->st) (void)hipStreamSynchronize(s->st);
    (void)hipFree(s->d_rec);
    (void)hipFree(s->d_loc);
    (void)hipFree(s->d_b64);
    (void)hipFree(s->d_x);
    (void)hipFree(s->d_side);
    (void)hipFree(s->d_x64);
    (void)hipFree(s->d_xref);
    (void)hipFree(s->d_part);
    (void)hipFree(s->d_scalar);
    (void)hipFree(s->d_trace);
    (void)hipFree(s->d_tau);
    if (s->h_pin) (void)hipHostFree(s->h_pin);
    if (s->e0) (void)hipEventDestroy(s->e0);
    if (s->e1) (void)hipEventDestroy(s->e1);
    delete s;
}

// Copy an input array to host memory if it lives on the device.
template <class T>
asyrk_status to_host(const asyrk_system *s, int mem, const T *src, size_t count, std::vector<T> &buf,
                     const T *&out) {
    if (mem == ASYRK_MEM_HOST || src == nullptr) {
        out = src;
        return ASYRK_OK;
    }
    try {
        buf.resize(count);
    } catch (...) {
        return ASYRK_ERR_OOM;
    }
    HIP_OK(hipMemcpy(buf.data(), src, count * sizeof(T), hipMemcpyDeviceToHost));
    out = buf.data();
    (void)s;
    return ASYRK_OK;
}

// Reduction to one device scalar, then to pinned host memory; synchronizes.
asyrk_status fetch_scalar(asyrk_system *s, int nparts, double *host_out) {
    HIP_OK(launch_finish_sum(s->d_part, nparts, s->d_scalar, s->st));
    HIP_OK(hipMemcpyAsync(s->h_pin, s->d_scalar, sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIP_OK(hipStreamSynchronize(s->st));
    *host_out = s->h_pin[0];
    return ASYRK_OK;
}

// Worker loops: 0 plain, 1 pipelined, 2 batched.
constexpr int kLoops = 3;
// Without autotuning, the batched worker loop is used up to kBatchMaxR
// workers and the pipelined one up to kPipeMaxR: below these the sweep is
// bound by each worker's memory latency (which the batched loop shortens
// most), above them by the atomic unit, where the plain loop measured faster.
constexpr int64_t kBatchMaxR = 1024;
constexpr int64_t kPipeMaxR = 8192;

// Lanes per row without autotuning: the sweep saturates once about 2^16
// lanes are in flight, so G is the largest power of two with R * G <= 2^16,
// but no wider than the smallest power of two covering the longest row's
// units (wider groups only idle) and at most 64.  Sized by the longest row,
// not the average: with few workers a long row read in several chunks costs a
// dependent round trip per chunk (heavy-tailed rows: 2-3x faster at G = 64
// than at the average's G = 8).  With so few workers that the covering
// groups would not give every CU a wave (R * G < 2^14 lanes), G grows until
// they do, idle lanes and all: spreading the workers over more CUs measured
// 7-8% faster at R = 512-1024 on 20-entry rows.  The single-coordinate
// update (Algorithm 1) issues one atomic per row and is bound by its gathers,
// which take twice the lanes in flight to saturate (R * G <= 2^17: 4.0e9
// against 3.2e9 rows/s at R = 65536 on 20-entry rows).
int auto_lanes(const asyrk_system *s, int64_t R, bool update_one) {
    const Geom g = geom_of(s->vk);
    const double units = (double)s->mu / g.U;
    const int64_t cap = (int64_t)1 << (update_one ? 17 : 16);
    int cover = 1;
    while (cover < 64 && cover < units) cover *= 2;
    int G = 1;
    while (G < cover && R * (2 * G) <= cap) G *= 2;
    while (G < 64 && R * G < ((int64_t)1 << 14)) G *= 2;
    return G;
}

// log2 of the iterate's element stride for an FP32 or FP64 iterate.  The
// single-coordinate update (Algorithm 1) issues one atomic per row against
// its gathers, so it is bound by gathers, which a dense iterate serves better
// from the caches: it uses the buffer densely.
int xshift_of(const asyrk_system *s, bool f32, const asyrk_solve_params &p) {
    if (p.update == ASYRK_UPDATE_ONE) return 0;
    return stride_shift(s->xstride, f32 ? 4 : 8);
}

double lambda_mp(const asyrk_system *s) {
    const double r = std::sqrt((double)s->n / (double)s->m);
    return (1.0 + r) * (1.0 + r) * s->fro2 / (double)s->n;
}

// Corollary 1: tau + 1 <= ||A||_F^2 / (2 e lambda_max), with lambda_max
// estimated by max(Gaussian-ensemble estimate, largest column norm^2); the
// latter is a lower bound that dominates for skewed (hot-column) matrices.
int64_t auto_in_flight(const asyrk_system *s) {
    const double lam = std::max(lambda_mp(s), s->max_col_norm2);
    const double tmax = std::floor(s->fro2 / (2.0 * M_E * lam));
    int64_t R = (int64_t)tmax;
    if (R < 1) R = 1;
    if (R > 65536) R = 65536;
    return R;
}

struct Monitor {
    bool use_ref = false;
    double ref_norm2 = 0.0;
    double b_norm2 = 0.0;
};

// Monitored error of an iterate on the device (x of the sweep dtype or FP64).
asyrk_status monitored_error(asyrk_system *s, const Monitor &mon, const void *x, int x_f32, int xsh, double *err) {
    double v = 0.0;
    if (mon.use_ref) {
        HIP_OK(launch_sumsq_diff(x, x_f32, xsh, s->d_xref, s->n, s->d_part, kResidualBlocks, s->st));
        asyrk_status rc = fetch_scalar(s, kResidualBlocks, &v);
        if (rc) return rc;
        *err = mon.ref_norm2 > 0 ? std::sqrt(v / mon.ref_norm2) : std::sqrt(v);
    } else {
        HIP_OK(launch_residual(s->vk, s->rows, s->d_b64, x, x_f32, xsh, nullptr, 0, s->d_part, kResidualBlocks, s->st));
        asyrk_status rc = fetch_scalar(s, kResidualBlocks, &v);
        if (rc) return rc;
        *err = mon.b_norm2 > 0 ? std::sqrt(v / mon.b_norm2) : std::sqrt(v);
    }
    return ASYRK_OK;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Staleness samples of the sweeps of one call, summed over launches.
struct TraceSums {
    double tau_max = 0.0, tau_sum = 0.0, count = 0.0, win_max = 0.0, win_sum = 0.0;
};
static asyrk_status run_sweeps(asyrk_system *s, const asyrk_solve_params &p, int xk, int G, int64_t R, double gamma,
                               uint64_t seed, int64_t t_begin, int64_t t_end, double *gpu_s, TraceSums *tr);
static asyrk_status create_from_device(asyrk_system **out, int64_t m, int64_t n, const int64_t *row_ptr,
                                       const int32_t *col, const void *vals, int32_t vals_dtype, const double *b,
                                       void *stream);
static asyrk_status create_from_host(asyrk_system **out, int64_t m, int64_t n, const int64_t *rp,
                                     const int32_t *cl, const uint8_t *vl, int32_t vals_dtype, const double *bb,
                                     int32_t mem, void *stream);

// =========================================================================

extern "C" {

int asyrk_abi_version(void) { return ASYRK_ABI_VERSION; }

const char *asyrk_status_string(asyrk_status s) {
    switch (s) {
        case ASYRK_OK: return "ok";
        case ASYRK_ERR_INVALID_ARG: return "invalid argument";
        case ASYRK_ERR_ZERO_ROW: return "A has a zero row";
        case ASYRK_ERR_OOM: return "out of memory";
        case ASYRK_ERR_DEVICE: return "HIP runtime error";
        case ASYRK_ERR_NOT_CONVERGED: return "tolerance not reached within the sweep budget";
        case ASYRK_ERR_DIVERGED: return "iteration diverged";
        case ASYRK_ERR_CANCELLED: return "cancelled";
        case ASYRK_ERR_UNSUPPORTED: return "unsupported combination";
        case ASYRK_PENDING: return "request pending";
        case ASYRK_ERR_SCRATCH: return "problem larger than the fixed scratch of an allocation-free entry point";
    }
    return "unknown status";
}

const char *asyrk_last_error_message(void) { return g_last; }

void asyrk_solve_params_init(asyrk_solve_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->mode = ASYRK_ASYNC;
    p->sampling = ASYRK_SAMPLE_NORM2;
    p->update = ASYRK_UPDATE_ALL;
    p->check_every = 1;
    p->iter_dtype = -1;
    p->pipeline = -1;
}

asyrk_status asyrk_create(asyrk_system **out, int64_t m, int64_t n, const int64_t *row_ptr,
                          const int32_t *col_idx, const void *vals, int32_t vals_dtype, const double *b,
                          int32_t mem, void *stream) {
    if (!out) return ASYRK_ERR_INVALID_ARG;
    *out = nullptr;
    if (mem != ASYRK_MEM_HOST && mem != ASYRK_MEM_DEVICE) return ASYRK_ERR_INVALID_ARG;
    if (m < 1 || n < 1 || m > INT32_MAX || n > INT32_MAX) return ASYRK_ERR_INVALID_ARG;
    if (vals_dtype != ASYRK_F64 && vals_dtype != ASYRK_F32 && vals_dtype != ASYRK_BF16)
        return ASYRK_ERR_INVALID_ARG;
    if (!row_ptr || !b) return ASYRK_ERR_INVALID_ARG;
    if (mem == ASYRK_MEM_DEVICE) return create_from_device(out, m, n, row_ptr, col_idx, vals, vals_dtype, b, stream);

    asyrk_system tmp_for_copy;
    std::vector<int64_t> rp_buf;
    std::vector<int32_t> col_buf;
    std::vector<uint8_t> val_buf;
    std::vector<double> b_buf;
    const int64_t *rp = nullptr;
    const int32_t *cl = nullptr;
    const uint8_t *vl = nullptr;
    const double *bb = nullptr;
    asyrk_status rc = to_host(&tmp_for_copy, mem, row_ptr, (size_t)m + 1, rp_buf, rp);
    if (rc) return rc;
    if (rp[0] != 0 || rp[m] < 0 || rp[m] >= INT32_MAX) return ASYRK_ERR_INVALID_ARG;
    const int64_t nnz = rp[m];
    const Geom g = geom_of(vals_dtype);
    if (nnz > 0 && (!col_idx || !vals)) return ASYRK_ERR_INVALID_ARG;
    rc = to_host(&tmp_for_copy, mem, col_idx, (size_t)nnz, col_buf, cl);
    if (rc) return rc;
    rc = to_host(&tmp_for_copy, mem, static_cast<const uint8_t *>(vals), (size_t)nnz * g.VB, val_buf, vl);
    if (rc) return rc;
    rc = to_host(&tmp_for_copy, mem, b, (size_t)m, b_buf, bb);
    if (rc) return rc;

    return create_from_host(out, m, n, rp, cl, vl, vals_dtype, bb, mem, stream);
}

// The device state of a system whose layout `res` describes; the records
// (rec_bytes), locators and b are left for the caller to fill.
static asyrk_status alloc_system(asyrk_system *&out, int64_t m, int64_t n, int32_t vals_dtype, int32_t mem,
                                 void *stream, const SetupResult &res, int64_t rec_bytes) {
    asyrk_system *s = new (std::nothrow) asyrk_system();
    if (!s) return ASYRK_ERR_OOM;
    s->m = m;
    s->n = n;
    s->nnz = res.nnz;
    s->vk = vals_dtype;
    s->mem = mem;
    s->st = (hipStream_t)stream;
    (void)hipGetDevice(&s->dev);
    s->mu = res.mu;
    s->nu = res.nu;
    s->fixed_nnz = res.fixed_nnz;
    s->stride = res.stride;
    s->fro2 = res.fro2;
    s->max_col_norm2 = res.max_col_norm2;
    s->rec_bytes = rec_bytes;

    hipError_t e = hipSuccess;
#define TRY(expr)                       \
    do {                                \
        e = (expr);                     \
        if (e != hipSuccess) goto fail; \
    } while (0)
    TRY(dmalloc(s, &s->d_rec, (size_t)rec_bytes));
    if (res.fixed_nnz == 0) TRY(dmalloc(s, &s->d_loc, res.loc.size() * sizeof(RowLoc)));
    TRY(dmalloc(s, &s->d_b64, (size_t)m * sizeof(double)));
    s->xstride = iterate_stride(n);
    TRY(dmalloc(s, &s->d_x, (size_t)n * (size_t)s->xstride));
    TRY(dmalloc(s, &s->d_x64, (size_t)n * sizeof(double)));
    TRY(dmalloc(s, &s->d_xref, (size_t)n * sizeof(double)));
    TRY(dmalloc(s, &s->d_part, (size_t)kResidualBlocks * sizeof(double)));
    TRY(dmalloc(s, &s->d_scalar, 4 * sizeof(double)));
    TRY(hipHostMalloc((void **)&s->h_pin, 4 * sizeof(double), hipHostMallocDefault));
    TRY(hipEventCreate(&s->e0));
    TRY(hipEventCreate(&s->e1));
#undef TRY
    s->rows.rec = s->d_rec;
    s->rows.loc = s->d_loc;
    s->rows.stride = s->stride;
    s->rows.fixed_nnz = (int32_t)s->fixed_nnz;
    s->rows.m = (int32_t)m;
    out = s;
    return ASYRK_OK;
fail:
    free_system(s);
    return dev_fail(e);
}

static asyrk_status create_from_host(asyrk_system **out, int64_t m, int64_t n, const int64_t *rp,
                                     const int32_t *cl, const uint8_t *vl, int32_t vals_dtype, const double *bb,
                                     int32_t mem, void *stream) {
    SetupResult res;
    asyrk_status rc = validate_system(m, n, rp, cl, vl, vals_dtype, bb, res);
    if (rc) return rc;
    rc = pack_records(m, rp, cl, vl, vals_dtype, bb, res);
    if (rc) return rc;
    asyrk_system *s = nullptr;
    rc = alloc_system(s, m, n, vals_dtype, mem, stream, res, (int64_t)res.rec.size());
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(s->d_rec, res.rec.data(), res.rec.size(), hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess && res.fixed_nnz == 0)
        e = hipMemcpyAsync(s->d_loc, res.loc.data(), res.loc.size() * sizeof(RowLoc), hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) e = hipMemcpyAsync(s->d_b64, bb, (size_t)m * sizeof(double), hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) {
        free_system(s);
        return dev_fail(e);
    }
    *out = s;
    return ASYRK_OK;
}

// Device temporaries of one call, freed when it returns.
struct DevScratch {
    std::vector<void *> ptrs;
    hipError_t alloc(void **p, size_t bytes) {
        hipError_t e = hipMalloc(p, bytes ? bytes : 16);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    ~DevScratch() {
        for (void *q : ptrs) (void)hipFree(q);
    }
};

// Inputs in device memory: row_ptr comes to the host (the record plan and the
// checks of the row boundaries), the entries are validated, weighed and
// packed on the device, and only the row weights make the round trip for the
// alias table.  Same statuses, records and statistics as the host path, the
// column norms up to rounding order.
static asyrk_status create_from_device(asyrk_system **out, int64_t m, int64_t n, const int64_t *row_ptr,
                                       const int32_t *col, const void *vals, int32_t vals_dtype, const double *b,
                                       void *stream) {
    const hipStream_t st = (hipStream_t)stream;
    SetupResult res;
    std::vector<int64_t> rp;
    try {
        rp.resize((size_t)m + 1);
        res.w.resize((size_t)m);
    } catch (...) {
        return ASYRK_ERR_OOM;
    }
    HIP_OK(hipMemcpyAsync(rp.data(), row_ptr, ((size_t)m + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (rp[0] != 0) return ASYRK_ERR_INVALID_ARG;
    int64_t mu = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (rp[i + 1] < rp[i]) return ASYRK_ERR_INVALID_ARG;
        mu = std::max(mu, rp[i + 1] - rp[i]);
    }
    const int64_t nnz = rp[m];
    if (nnz >= (int64_t)INT32_MAX) return ASYRK_ERR_INVALID_ARG;
    if (nnz > 0 && (!col || !vals)) return ASYRK_ERR_INVALID_ARG;

    DevScratch tmp;
    double *d_w = nullptr, *d_sq = nullptr;
    uint32_t *d_cnt = nullptr;
    unsigned long long *d_misc = nullptr;  // flags, max column count, bits of the max column norm
    HIP_OK(tmp.alloc((void **)&d_w, (size_t)m * sizeof(double)));
    HIP_OK(tmp.alloc((void **)&d_cnt, (size_t)n * sizeof(uint32_t)));
    HIP_OK(tmp.alloc((void **)&d_sq, (size_t)n * sizeof(double)));
    HIP_OK(tmp.alloc((void **)&d_misc, 3 * sizeof(unsigned long long)));
    HIP_OK(hipMemsetAsync(d_cnt, 0, (size_t)n * sizeof(uint32_t), st));
    HIP_OK(hipMemsetAsync(d_sq, 0, (size_t)n * sizeof(double), st));
    HIP_OK(hipMemsetAsync(d_misc, 0, 3 * sizeof(unsigned long long), st));
    HIP_OK(launch_scan_rows_dev(vals_dtype, m, n, row_ptr, col, vals, b, d_w, d_cnt, d_sq, (uint32_t *)d_misc, st));
    HIP_OK(launch_col_max_dev(d_cnt, d_sq, n, d_misc + 1, st));
    unsigned long long misc[3] = {0, 0, 0};
    HIP_OK(hipMemcpyAsync(res.w.data(), d_w, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(misc, d_misc, sizeof misc, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if ((uint32_t)misc[0] != 0) return ASYRK_ERR_INVALID_ARG;
    for (int64_t i = 0; i < m; ++i)
        if (!(res.w[i] > 0.0)) return ASYRK_ERR_ZERO_ROW;

    res.nnz = nnz;
    res.mu = mu;
    res.nu = (int64_t)misc[1];
    std::memcpy(&res.max_col_norm2, &misc[2], sizeof(double));
    res.fixed_nnz = rp[1] - rp[0];
    for (int64_t i = 1; i < m && res.fixed_nnz > 0; ++i)
        if (rp[i + 1] - rp[i] != res.fixed_nnz) res.fixed_nnz = 0;
    double fro2 = 0.0;
    for (int64_t i = 0; i < m; ++i) fro2 = fro2 + res.w[i];
    res.fro2 = fro2;
    int64_t total = 0;
    asyrk_status rc = plan_records(m, rp.data(), vals_dtype, res, &total);
    if (rc) return rc;

    std::unique_ptr<RowAux[]> aux(new (std::nothrow) RowAux[m]);
    {
        std::unique_ptr<uint32_t[]> thresh(new (std::nothrow) uint32_t[m]);
        std::unique_ptr<int32_t[]> alias(new (std::nothrow) int32_t[m]);
        if (!aux || !thresh || !alias) return ASYRK_ERR_OOM;
        build_alias(res.w.data(), m, res.fro2, thresh.get(), alias.get());
        row_aux(res.w.data(), m, thresh.get(), alias.get(), aux.get());
    }
    RowAux *d_aux = nullptr;
    HIP_OK(tmp.alloc((void **)&d_aux, (size_t)m * sizeof(RowAux)));
    HIP_OK(hipMemcpyAsync(d_aux, aux.get(), (size_t)m * sizeof(RowAux), hipMemcpyHostToDevice, st));

    asyrk_system *s = nullptr;
    rc = alloc_system(s, m, n, vals_dtype, ASYRK_MEM_DEVICE, stream, res, total);
    if (rc) return rc;
    hipError_t e = hipSuccess;
    if (res.fixed_nnz == 0)
        e = hipMemcpyAsync(s->d_loc, res.loc.data(), res.loc.size() * sizeof(RowLoc), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_write_records_dev(vals_dtype, m, row_ptr, col, vals, b, d_aux, res.stride,
                                     res.fixed_nnz == 0 ? s->d_loc : nullptr, s->d_rec, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s->d_b64, b, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_system(s);
        return dev_fail(e);
    }
    *out = s;
    return ASYRK_OK;
}

asyrk_status asyrk_records_get(asyrk_system *s, void *dst, int64_t cap, int64_t *bytes_out) {
    if (!s) return ASYRK_ERR_INVALID_ARG;
    if (bytes_out) *bytes_out = s->rec_bytes;
    if (!dst) return ASYRK_OK;
    if (cap < s->rec_bytes) return ASYRK_ERR_INVALID_ARG;
    if (s->rec_b_dirty) {  // a refinement left its residual in the headers
        HIP_OK(launch_set_rec_b(s->vk, s->rows, s->d_b64, s->st));
        s->rec_b_dirty = false;
    }
    HIP_OK(hipStreamSynchronize(s->st));
    HIP_OK(hipMemcpy(dst, s->d_rec, (size_t)s->rec_bytes, hipMemcpyDeviceToHost));
    return ASYRK_OK;
}

asyrk_status asyrk_destroy(asyrk_system *s) {
    free_system(s);
    return ASYRK_OK;
}

asyrk_status asyrk_create_augmented(asyrk_system **out, int64_t m, int64_t n, const int64_t *row_ptr,
                                    const int32_t *col_idx, const void *vals, int32_t vals_dtype, const double *b,
                                    double zeta, double phi, int32_t mem, void *stream) {
    if (!out) return ASYRK_ERR_INVALID_ARG;
    *out = nullptr;
    if (mem != ASYRK_MEM_HOST && mem != ASYRK_MEM_DEVICE) return ASYRK_ERR_INVALID_ARG;
    if (m < 1 || n < 1 || m > INT32_MAX || n > INT32_MAX) return ASYRK_ERR_INVALID_ARG;
    if (vals_dtype != ASYRK_F64 && vals_dtype != ASYRK_F32 && vals_dtype != ASYRK_BF16)
        return ASYRK_ERR_INVALID_ARG;
    if (!row_ptr || !b || !col_idx || !vals) return ASYRK_ERR_INVALID_ARG;
    asyrk_system tmp_for_copy;
    std::vector<int64_t> rp_buf;
    std::vector<int32_t> col_buf;
    std::vector<uint8_t> val_buf;
    std::vector<double> b_buf;
    const int64_t *rp = nullptr;
    const int32_t *cl = nullptr;
    const uint8_t *vl = nullptr;
    const double *bb = nullptr;
    asyrk_status rc = to_host(&tmp_for_copy, mem, row_ptr, (size_t)m + 1, rp_buf, rp);
    if (rc) return rc;
    if (rp[0] != 0 || rp[m] < 0 || rp[m] >= INT32_MAX) return ASYRK_ERR_INVALID_ARG;
    const Geom g = geom_of(vals_dtype);
    rc = to_host(&tmp_for_copy, mem, col_idx, (size_t)rp[m], col_buf, cl);
    if (rc) return rc;
    rc = to_host(&tmp_for_copy, mem, static_cast<const uint8_t *>(vals), (size_t)rp[m] * g.VB, val_buf, vl);
    if (rc) return rc;
    rc = to_host(&tmp_for_copy, mem, b, (size_t)m, b_buf, bb);
    if (rc) return rc;
    SetupResult chk;  // A itself must be a valid CSR with no zero row
    rc = validate_system(m, n, rp, cl, vl, vals_dtype, bb, chk);
    if (rc) return rc;
    AugCSR aug;
    rc = build_augmented(m, n, rp, cl, vl, vals_dtype, bb, zeta, phi, aug);
    if (rc) return rc;
    rc = create_from_host(out, n + m, n + m, aug.row_ptr.data(), aug.col.data(), aug.vals.data(), vals_dtype,
                          aug.b.data(), mem, stream);
    if (rc) return rc;
    (*out)->aug_n = n;
    (*out)->aug_zeta = zeta;
    return ASYRK_OK;
}

asyrk_status asyrk_augmented_solution(asyrk_system *s, const double *z, double *x_out) {
    if (!s || !z || !x_out || s->aug_n <= 0) return ASYRK_ERR_INVALID_ARG;
    const size_t bytes = (size_t)s->aug_n * sizeof(double);
    if (s->mem == ASYRK_MEM_DEVICE) {
        HIP_OK(launch_divide(z, s->aug_zeta, x_out, s->aug_n, s->st));
    } else {
        HIP_OK(hipMemcpyAsync(s->d_x64, z, bytes, hipMemcpyHostToDevice, s->st));
        HIP_OK(launch_divide(s->d_x64, s->aug_zeta, s->d_x64, s->aug_n, s->st));
        HIP_OK(hipMemcpyAsync(x_out, s->d_x64, bytes, hipMemcpyDeviceToHost, s->st));
    }
    HIP_OK(hipStreamSynchronize(s->st));
    return ASYRK_OK;
}

asyrk_status asyrk_system_info_get(const asyrk_system *s, asyrk_system_info *info) {
    if (!s || !info) return ASYRK_ERR_INVALID_ARG;
    std::memset(info, 0, sizeof *info);
    info->m = s->m;
    info->n = s->n;
    info->nnz = s->nnz;
    info->mu = s->mu;
    info->nu = s->nu;
    info->fixed_nnz = s->fixed_nnz;
    info->record_stride = s->stride;
    info->device_bytes = s->device_bytes;
    info->vals_dtype = s->vk;
    info->iter_dtype = ASYRK_F64;
    info->fro2 = s->fro2;
    info->lambda_mp = lambda_mp(s);
    const Geom g = geom_of(s->vk);
    const int sc = s->vk == ASYRK_F64 ? 8 : 4;  // b_i and w_i in the sweep dtype, 4-byte start
    info->record_bytes_per_row =
        (int64_t)std::llround((double)s->nnz / (double)s->m * (4 + g.VB)) + 2 * sc + 4;
    info->max_col_norm2 = s->max_col_norm2;
    info->default_in_flight = auto_in_flight(s);
    info->iterate_stride = s->xstride;
    info->tuned_in_flight = s->tuned_auto_R[0] ? s->tuned_R[0] : 0;
    return ASYRK_OK;
}

asyrk_status asyrk_set_rhs(asyrk_system *s, const double *b) {
    if (!s || !b) return ASYRK_ERR_INVALID_ARG;
    if (s->mem == ASYRK_MEM_DEVICE) {
        // checked where it lies; only the verdict comes to the host
        DevScratch tmp;
        uint32_t *d_flag = nullptr;
        HIP_OK(tmp.alloc((void **)&d_flag, sizeof(uint32_t)));
        HIP_OK(hipMemsetAsync(d_flag, 0, sizeof(uint32_t), s->st));
        HIP_OK(launch_check_finite_dev(b, s->m, d_flag, s->st));
        HIP_OK(hipMemcpyAsync(s->h_pin, d_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s->st));
        HIP_OK(hipStreamSynchronize(s->st));
        uint32_t flag = 0;
        std::memcpy(&flag, s->h_pin, sizeof flag);
        if (flag) return ASYRK_ERR_INVALID_ARG;
        HIP_OK(hipMemcpyAsync(s->d_b64, b, (size_t)s->m * sizeof(double), hipMemcpyDeviceToDevice, s->st));
    } else {
        for (int64_t i = 0; i < s->m; ++i)
            if (!std::isfinite(b[i])) return ASYRK_ERR_INVALID_ARG;
        HIP_OK(hipMemcpyAsync(s->d_b64, b, (size_t)s->m * sizeof(double), hipMemcpyHostToDevice, s->st));
    }
    HIP_OK(launch_set_rec_b(s->vk, s->rows, s->d_b64, s->st));
    if (s->d_side) HIP_OK(launch_build_side(s->vk, s->rows, s->d_b64, s->d_side, s->st));
    HIP_OK(hipStreamSynchronize(s->st));
    s->rec_b_dirty = false;
    return ASYRK_OK;
}

asyrk_status asyrk_residual(asyrk_system *s, const double *x, double *r_out, double *norm2_out) {
    if (!s || !x || !norm2_out) return ASYRK_ERR_INVALID_ARG;
    const hipMemcpyKind h2d = s->mem == ASYRK_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HIP_OK(hipMemcpyAsync(s->d_x64, x, (size_t)s->n * sizeof(double), h2d, s->st));
    double *r_dev = nullptr;
    if (r_out) {
        if (s->mem == ASYRK_MEM_DEVICE)
            r_dev = r_out;
        else
            HIP_OK(hipMalloc((void **)&r_dev, (size_t)s->m * sizeof(double)));
    }
    hipError_t e = launch_residual(s->vk, s->rows, s->d_b64, s->d_x64, 0, 0, r_dev, 0, s->d_part,
                                   kResidualBlocks, s->st);
    double v = 0.0;
    asyrk_status rc = e == hipSuccess ? fetch_scalar(s, kResidualBlocks, &v) : dev_fail(e);
    if (rc == ASYRK_OK && r_out && s->mem == ASYRK_MEM_HOST) {
        e = hipMemcpy(r_out, r_dev, (size_t)s->m * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = dev_fail(e);
    }
    if (r_dev && s->mem == ASYRK_MEM_HOST) (void)hipFree(r_dev);
    if (rc == ASYRK_OK) *norm2_out = v;
    return rc;
}

asyrk_status asyrk_sample_rows(asyrk_system *s, uint64_t seed, uint32_t stream_id, int32_t sampling,
                               int64_t ticket0, int64_t count, int32_t *rows_out, int32_t *coords_out) {
    if (!s || !rows_out || count < 0 || ticket0 < 0) return ASYRK_ERR_INVALID_ARG;
    if (sampling != ASYRK_SAMPLE_NORM2 && sampling != ASYRK_SAMPLE_UNIFORM) return ASYRK_ERR_INVALID_ARG;
    if (count == 0) return ASYRK_OK;
    int32_t *dr = rows_out, *dc = coords_out;
    const bool host = s->mem == ASYRK_MEM_HOST;
    if (host) {
        HIP_OK(hipMalloc((void **)&dr, (size_t)count * 4 * 2));
        dc = coords_out ? dr + count : nullptr;
    }
    hipError_t e = launch_sample_rows(s->vk, s->rows, ticket0, count, (uint32_t)seed, (uint32_t)(seed >> 32),
                                      stream_id, sampling == ASYRK_SAMPLE_UNIFORM, dr, dc, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e == hipSuccess && host) {
        e = hipMemcpy(rows_out, dr, (size_t)count * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && coords_out) e = hipMemcpy(coords_out, dc, (size_t)count * 4, hipMemcpyDeviceToHost);
    }
    if (host) (void)hipFree(dr);
    return e == hipSuccess ? ASYRK_OK : dev_fail(e);
}

asyrk_status asyrk_lambda_max(asyrk_system *s, int32_t iters, uint64_t seed, double *lambda_out,
                              double *tau_max_out) {
    if (!s || !lambda_out || iters < 1) return ASYRK_ERR_INVALID_ARG;
    double *v = nullptr, *z = nullptr, *y = nullptr;
    HIP_OK(hipMalloc((void **)&v, (size_t)s->n * 8));
    hipError_t e = hipMalloc((void **)&z, (size_t)s->n * 8);
    if (e == hipSuccess) e = hipMalloc((void **)&y, (size_t)s->m * 8);
    double lam = 0.0, nrm2 = 0.0;
    asyrk_status rc = ASYRK_OK;
    if (e == hipSuccess) e = launch_random_fill(v, s->n, (uint32_t)seed, (uint32_t)(seed >> 32), s->st);
    // v <- v / ||v||
    if (e == hipSuccess) e = launch_sumsq_diff(v, 0, 0, nullptr, s->n, s->d_part, kResidualBlocks, s->st);
    if (e == hipSuccess) e = launch_finish_sum(s->d_part, kResidualBlocks, s->d_scalar, s->st);
    if (e == hipSuccess) e = launch_scale(v, s->n, s->d_scalar, s->st);
    for (int it = 0; it < iters && e == hipSuccess; ++it) {
        // y = -A v (residual with b = 0), z = A^T y, v = z / ||z||
        e = launch_residual(s->vk, s->rows, nullptr, v, 0, 0, y, 0, s->d_part, kResidualBlocks, s->st);
        if (e == hipSuccess) e = launch_zero(z, s->n * 8, s->st);
        if (e == hipSuccess) e = launch_scatter_rows(s->vk, s->rows, y, z, s->st);
        if (e == hipSuccess) e = launch_sumsq_diff(z, 0, 0, nullptr, s->n, s->d_part, kResidualBlocks, s->st);
        if (e == hipSuccess) e = launch_finish_sum(s->d_part, kResidualBlocks, s->d_scalar, s->st);
        if (e == hipSuccess) e = launch_scale(z, s->n, s->d_scalar, s->st);
        if (e == hipSuccess) std::swap(v, z);
    }
    // Rayleigh quotient ||A v||^2 with ||v|| = 1
    if (e == hipSuccess)
        e = launch_residual(s->vk, s->rows, nullptr, v, 0, 0, nullptr, 0, s->d_part, kResidualBlocks, s->st);
    if (e == hipSuccess) {
        rc = fetch_scalar(s, kResidualBlocks, &nrm2);
        lam = nrm2;
    }
    (void)hipFree(v);
    (void)hipFree(z);
    (void)hipFree(y);
    if (e != hipSuccess) return dev_fail(e);
    if (rc) return rc;
    *lambda_out = lam;
    if (lam > 0.0 && std::isfinite(lam)) s->lambda_pi = lam;
    if (tau_max_out) {
        const double t = std::floor(s->fro2 / (2.0 * M_E * lam)) - 1.0;
        *tau_max_out = t >= 0 ? t : -1.0;
    }
    return ASYRK_OK;
}

// ------------------------------------------------------- allocation-free lambda_max
//
// Scratch of asyrk_lambda_max_noalloc: the power iteration's vectors v, z (n
// doubles each) and y (m doubles), the reduction partials and one device
// scalar.  A file-scope device array, so that the entry point allocates
// nothing; every device the library runs on holds one copy for the life of
// the process.  In host code `scratch` names a host-side stand-in: its device
// address on each device comes from hipGetSymbolAddress (scratch_on).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};  // per device, looked up once with that device current

// The device address of `scratch` on the current device (looked up once).
hipError_t scratch_on(int dev, uint8_t **out) {
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<uint8_t *>(g_scratch_ptr[dev]);
    return hipSuccess;
}

}  // namespace

asyrk_status asyrk_lambda_max_noalloc(asyrk_system *s, int32_t iters, uint64_t seed, double *lambda_out,
                                      double *tau_max_out) {
    if (!s || !lambda_out || iters < 1) return ASYRK_ERR_INVALID_ARG;
    const size_t need = (2 * (size_t)s->n + (size_t)s->m + (size_t)kResidualBlocks + 1) * sizeof(double);
    if (need > kNoAllocScratchBytes) {
        g_last = "asyrk_lambda_max_noalloc: 2 n + m + 2049 doubles exceed the 64 MiB scratch";
        return ASYRK_ERR_SCRATCH;
    }
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != s->dev) {
        g_last = "asyrk_lambda_max_noalloc: the system's device is not the current device";
        return ASYRK_ERR_INVALID_ARG;
    }
    uint8_t *base = nullptr;
    HIP_OK(scratch_on(dev, &base));
    double *v = reinterpret_cast<double *>(base);
    double *z = v + s->n;
    double *y = z + s->n;
    double *part = y + s->m;
    double *scal = part + kResidualBlocks;
    const hipStream_t st = s->st;
    // the same steps as asyrk_lambda_max, on scratch instead of fresh buffers
    HIP_OK(launch_random_fill(v, s->n, (uint32_t)seed, (uint32_t)(seed >> 32), st));
    HIP_OK(launch_sumsq_diff(v, 0, 0, nullptr, s->n, part, kResidualBlocks, st));
    HIP_OK(launch_finish_sum(part, kResidualBlocks, scal, st));
    HIP_OK(launch_scale(v, s->n, scal, st));
    for (int it = 0; it < iters; ++it) {
        HIP_OK(launch_residual(s->vk, s->rows, nullptr, v, 0, 0, y, 0, part, kResidualBlocks, st));
        HIP_OK(launch_zero(z, s->n * 8, st));
        HIP_OK(launch_scatter_rows(s->vk, s->rows, y, z, st));
        HIP_OK(launch_sumsq_diff(z, 0, 0, nullptr, s->n, part, kResidualBlocks, st));
        HIP_OK(launch_finish_sum(part, kResidualBlocks, scal, st));
        HIP_OK(launch_scale(z, s->n, scal, st));
        std::swap(v, z);
    }
    HIP_OK(launch_residual(s->vk, s->rows, nullptr, v, 0, 0, nullptr, 0, part, kResidualBlocks, st));
    HIP_OK(launch_finish_sum(part, kResidualBlocks, scal, st));
    HIP_OK(hipMemcpyAsync(s->h_pin, scal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const double lam = s->h_pin[0];
    *lambda_out = lam;
    if (lam > 0.0 && std::isfinite(lam)) s->lambda_pi = lam;
    if (tau_max_out) {
        const double t = std::floor(s->fro2 / (2.0 * M_E * lam)) - 1.0;
        *tau_max_out = t >= 0 ? t : -1.0;
    }
    return ASYRK_OK;
}

// Time every lane-group width and worker loop at R workers; returns the
// chosen pair and its rate (the near-tie rule below) and the rates of all 21.
static asyrk_status tune_at(asyrk_system *s, int xk, int64_t R, double gamma, int *G_out, int *pipe_out,
                            double *rate_out, double *rates21) {
    asyrk_solve_params p;
    asyrk_solve_params_init(&p);
    // at least one sweep and at least 2M tickets per candidate
    const int64_t tickets = std::max<int64_t>(s->m, (int64_t)2 << 20);
    const int cands[7] = {1, 2, 4, 8, 16, 32, 64};
    double rate[kLoops][7] = {}, top[kLoops] = {};
    for (int pipe = 0; pipe < kLoops; ++pipe) {
        p.pipeline = pipe;
        for (int k = 0; k < 7; ++k) {
            const int G = cands[k];
            HIP_OK(launch_zero(s->d_x, s->n * s->xstride, s->st));
            double gpu_s = 0.0;
            TraceSums unused;
            asyrk_status rc = run_sweeps(s, p, xk, G, R, gamma, 0x5eedull, 0, tickets, &gpu_s, &unused);
            if (rc) return rc;
            rate[pipe][k] = gpu_s > 0 ? (double)tickets / gpu_s : 0.0;
            top[pipe] = std::max(top[pipe], rate[pipe][k]);
            if (rates21) rates21[7 * pipe + k] = rate[pipe][k];
        }
    }
    // Candidates a few percent apart differ by timing noise (a saturated
    // atomic unit), so ties are broken by a fixed rule: a loop replaces the
    // one chosen so far (plain, then pipelined, then batched) only when it is
    // more than 3% faster, then the narrowest lane group within 3% of that
    // loop's fastest.
    int best_pipe = 0;
    for (int pipe = 1; pipe < kLoops; ++pipe)
        if (top[pipe] > 1.03 * top[best_pipe]) best_pipe = pipe;
    int k_best = 6;
    for (int k = 0; k < 7; ++k)
        if (rate[best_pipe][k] >= 0.97 * top[best_pipe]) {
            k_best = k;
            break;
        }
    *G_out = cands[k_best];
    *pipe_out = best_pipe;
    *rate_out = rate[best_pipe][k_best];
    return ASYRK_OK;
}

asyrk_status asyrk_autotune(asyrk_system *s, double gamma, int32_t iter_dtype, int64_t in_flight,
                            int32_t *best_lanes, int32_t *best_pipeline, double *rows_per_s_out) {
    if (!s || !(gamma > 0.0 && gamma < 2.0) || in_flight < -1) return ASYRK_ERR_INVALID_ARG;
    if (iter_dtype != -1 && iter_dtype != ASYRK_F32 && iter_dtype != ASYRK_F64) return ASYRK_ERR_INVALID_ARG;
    const int xk = iter_dtype >= 0 ? iter_dtype : ASYRK_F64;
    if (s->vk == ASYRK_F64 && xk == ASYRK_F32) return ASYRK_ERR_UNSUPPORTED;
    if (s->rec_b_dirty) {
        HIP_OK(launch_set_rec_b(s->vk, s->rows, s->d_b64, s->st));
        s->rec_b_dirty = false;
    }
    if (xk == ASYRK_F64 && s->vk != ASYRK_F64 && !s->d_side) {
        HIP_OK(dmalloc(s, &s->d_side, (size_t)s->m * sizeof(double2)));
        HIP_OK(launch_build_side(s->vk, s->rows, s->d_b64, s->d_side, s->st));
    }
    const int64_t R_max = auto_in_flight(s);
    int G = 0, pipe = 0;
    double r_best = 0.0;
    int64_t R = in_flight > 0 ? in_flight : R_max;
    if (in_flight == -1) {
        // The in-flight count too: powers of two from 1024 up to Corollary 1's
        // bound, and the bound itself.  The smallest R within 2% of the
        // fastest wins: the same throughput with less staleness.
        std::vector<int64_t> Rs;
        for (int64_t r = 1024; r < R_max; r *= 2) Rs.push_back(r);
        Rs.push_back(R_max);
        std::vector<double> rr(Rs.size(), 0.0);
        std::vector<int> gg(Rs.size(), 0), pp(Rs.size(), 0);
        double top = 0.0;
        for (size_t k = 0; k < Rs.size(); ++k) {
            asyrk_status rc = tune_at(s, xk, Rs[k], gamma, &gg[k], &pp[k], &rr[k], nullptr);
            if (rc) return rc;
            top = std::max(top, rr[k]);
        }
        size_t kb = Rs.size() - 1;
        for (size_t k = 0; k < Rs.size(); ++k)
            if (rr[k] >= 0.98 * top) {
                kb = k;
                break;
            }
        R = Rs[kb];
    }
    // the chosen R's candidates, timed again for the reported rates
    asyrk_status rc = tune_at(s, xk, R, gamma, &G, &pipe, &r_best, rows_per_s_out);
    if (rc) return rc;
    const int xi = xk == ASYRK_F32 ? 1 : 0;
    s->tuned_G[xi] = G;
    s->tuned_pipe[xi] = pipe;
    s->tuned_R[xi] = R;
    s->tuned_auto_R[xi] = in_flight == -1;
    if (best_lanes) *best_lanes = G;
    if (best_pipeline) *best_pipeline = pipe;
    return ASYRK_OK;
}

asyrk_status asyrk_probe_copy(int64_t bytes, int32_t iters, double *gbps) {
    if (bytes < 16 || iters < 1 || !gbps) return ASYRK_ERR_INVALID_ARG;
    HIP_OK(probe_copy(bytes, iters, gbps));
    return ASYRK_OK;
}

asyrk_status asyrk_probe_scatter(int64_t n, int64_t count, int32_t dtype, int32_t kind, int32_t iters,
                                 double *per_s) {
    if (n < 1 || n > INT32_MAX || count < 1 || iters < 1 || !per_s) return ASYRK_ERR_INVALID_ARG;
    if ((dtype != ASYRK_F32 && dtype != ASYRK_F64) || (kind != 0 && kind != 1)) return ASYRK_ERR_INVALID_ARG;
    HIP_OK(probe_scatter(n, count, dtype, kind, iters, per_s));
    return ASYRK_OK;
}

// ------------------------------------------------------------------- solve

static asyrk_status run_sweeps(asyrk_system *s, const asyrk_solve_params &p, int xk, int G, int64_t R, double gamma,
                               uint64_t seed, int64_t t_begin, int64_t t_end, double *gpu_s, TraceSums *tr) {
    SweepArgs a{};
    a.rows = s->rows;
    a.x = s->d_x;
    a.xshift = xshift_of(s, xk == ASYRK_F32, p);
    a.side = s->d_side;
    a.t_begin = t_begin;
    a.t_end = t_end;
    a.R = R;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.stream_id = p.stream_id;
    a.uniform = p.sampling == ASYRK_SAMPLE_UNIFORM;
    a.update_one = p.update == ASYRK_UPDATE_ONE;
    a.replay = p.mode == ASYRK_REPLAY;
    a.gamma = gamma;
    a.trace = p.trace ? s->d_trace : nullptr;
    a.tau_ctr = p.trace ? s->d_tau : nullptr;
    a.slices = p.order;
    a.pipe = p.pipeline;
    const int64_t waves = (R * G + 63) / 64;
    if (p.trace) HIP_OK(launch_zero(s->d_trace, waves * kTraceWords * 8, s->st));
    HIP_OK(hipEventRecord(s->e0, s->st));
    if (p.order == 1)
        HIP_OK(launch_sweep_slices(s->vk, xk, G, a, s->st));
    else
        HIP_OK(launch_sweep(s->vk, xk, G, a, s->st));
    HIP_OK(hipEventRecord(s->e1, s->st));
    HIP_OK(hipEventSynchronize(s->e1));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, s->e0, s->e1));
    *gpu_s += ms * 1e-3;
    if (p.trace) {
        std::vector<uint64_t> w((size_t)waves * kTraceWords);
        HIP_OK(hipMemcpy(w.data(), s->d_trace, w.size() * 8, hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < waves; ++k) {
            const uint64_t *o = w.data() + k * kTraceWords;
            tr->tau_max = std::max(tr->tau_max, (double)o[0]);
            tr->tau_sum += (double)o[1];
            tr->count += (double)o[2];
            tr->win_max = std::max(tr->win_max, (double)o[3]);
            tr->win_sum += (double)o[4];
        }
    }
    return ASYRK_OK;
}

asyrk_status asyrk_solve(asyrk_system *s, double *x, double gamma, int64_t sweeps, uint64_t seed,
                         const asyrk_solve_params *pin, asyrk_solve_stats *st) {
    const double wall0 = now_s();
    if (!s || !x) return ASYRK_ERR_INVALID_ARG;
    asyrk_solve_params p;
    if (pin)
        p = *pin;
    else
        asyrk_solve_params_init(&p);
    if (!(gamma > 0.0 && gamma < 2.0) || sweeps < 0) return ASYRK_ERR_INVALID_ARG;
    if (p.mode != ASYRK_ASYNC && p.mode != ASYRK_REPLAY) return ASYRK_ERR_INVALID_ARG;
    if (p.sampling != ASYRK_SAMPLE_NORM2 && p.sampling != ASYRK_SAMPLE_UNIFORM) return ASYRK_ERR_INVALID_ARG;
    if (p.update != ASYRK_UPDATE_ALL && p.update != ASYRK_UPDATE_ONE) return ASYRK_ERR_INVALID_ARG;
    if (p.lanes != 0 && p.lanes != 1 && p.lanes != 2 && p.lanes != 4 && p.lanes != 8 && p.lanes != 16 &&
        p.lanes != 32 && p.lanes != 64)
        return ASYRK_ERR_INVALID_ARG;
    if (p.in_flight < 0 || p.check_every < 1 || !(p.tol >= 0.0) || !std::isfinite(p.tol) || p.ticket0 < 0 ||
        p.inner_sweeps < 0 || p.history_cap < 0 || (p.history_cap > 0 && !p.history))
        return ASYRK_ERR_INVALID_ARG;
    if (p.order != 0 && p.order != 1) return ASYRK_ERR_INVALID_ARG;
    if (p.pipeline < -1 || p.pipeline > 2 || (p.skip_resid != 0 && p.skip_resid != 1)) return ASYRK_ERR_INVALID_ARG;
    if (p.pipeline >= 1 && (p.mode != ASYRK_ASYNC || p.update != ASYRK_UPDATE_ALL)) return ASYRK_ERR_UNSUPPORTED;
    if (p.order == 1 && p.update != ASYRK_UPDATE_ALL) return ASYRK_ERR_UNSUPPORTED;
    if (p.order == 1 && p.ticket0 % s->m != 0) return ASYRK_ERR_INVALID_ARG;
    if (p.iter_dtype != -1 && p.iter_dtype != ASYRK_F32 && p.iter_dtype != ASYRK_F64) return ASYRK_ERR_INVALID_ARG;
    // FP64 by default: FP64 atomics outrun FP32 ones on this part, so the FP64
    // iterate is both faster and more accurate; refinement sweeps in FP32
    const int xk = p.iter_dtype >= 0 ? p.iter_dtype : (p.refine ? ASYRK_F32 : ASYRK_F64);
    if (s->vk == ASYRK_F64 && xk == ASYRK_F32) return ASYRK_ERR_UNSUPPORTED;
    if (p.refine && xk == ASYRK_F64) return ASYRK_ERR_UNSUPPORTED;
    if (p.refine && (p.mode == ASYRK_REPLAY || p.update == ASYRK_UPDATE_ONE)) return ASYRK_ERR_UNSUPPORTED;
    if (sweeps > (INT64_MAX - p.ticket0) / s->m) return ASYRK_ERR_INVALID_ARG;

    const int xi = xk == ASYRK_F32 ? 1 : 0;
    // an R the autotuner chose holds for the solves it timed: asynchronous,
    // all-coordinate, with replacement (traced or not)
    const bool tuned_kind = p.mode == ASYRK_ASYNC && p.update == ASYRK_UPDATE_ALL && p.order == 0;
    int64_t R = p.mode == ASYRK_REPLAY ? 1
                : p.in_flight          ? p.in_flight
                : (tuned_kind && s->tuned_auto_R[xi]) ? s->tuned_R[xi]
                                                      : auto_in_flight(s);
    // the autotuned pair holds at the R and for the kind of solve it was measured on
    const int tuned = tuned_kind && s->tuned_R[xi] == R ? s->tuned_G[xi] : 0;
    const int G = p.lanes ? p.lanes : (tuned ? tuned : auto_lanes(s, R, p.update == ASYRK_UPDATE_ONE));
    if (R > ((int64_t)1 << 26)) return ASYRK_ERR_INVALID_ARG;
    if (p.pipeline == -1) {
        const bool allowed = p.mode == ASYRK_ASYNC && p.update == ASYRK_UPDATE_ALL;
        const bool tuned_here = tuned && G == tuned;
        p.pipeline = !allowed ? 0
                     : (tuned_here ? s->tuned_pipe[xi] : (R <= kBatchMaxR ? 2 : (R <= kPipeMaxR ? 1 : 0)));
    }
    const bool f32 = xk == ASYRK_F32;
    const int xsh = xshift_of(s, f32, p);
    const hipMemcpyKind h2d = s->mem == ASYRK_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const hipMemcpyKind d2h = s->mem == ASYRK_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;

    asyrk_solve_stats S;
    std::memset(&S, 0, sizeof S);
    S.final_err = NAN;
    S.in_flight = R;
    S.lanes = G;
    S.pipelined = p.pipeline;
    S.tau_design = (double)(R - 1);

    // inputs
    HIP_OK(hipMemcpyAsync(s->d_x64, x, (size_t)s->n * 8, h2d, s->st));
    Monitor mon;
    if (p.x_ref) {
        mon.use_ref = true;
        HIP_OK(hipMemcpyAsync(s->d_xref, p.x_ref, (size_t)s->n * 8, h2d, s->st));
        HIP_OK(launch_sumsq_diff(s->d_xref, 0, 0, nullptr, s->n, s->d_part, kResidualBlocks, s->st));
        asyrk_status rc = fetch_scalar(s, kResidualBlocks, &mon.ref_norm2);
        if (rc) return rc;
    } else {
        HIP_OK(launch_sumsq_diff(s->d_b64, 0, 0, nullptr, s->m, s->d_part, kResidualBlocks, s->st));
        asyrk_status rc = fetch_scalar(s, kResidualBlocks, &mon.b_norm2);
        if (rc) return rc;
    }
    if (s->rec_b_dirty) {
        HIP_OK(launch_set_rec_b(s->vk, s->rows, s->d_b64, s->st));
        s->rec_b_dirty = false;
    }
    if (xk == ASYRK_F64 && s->vk != ASYRK_F64 && !s->d_side) {
        HIP_OK(dmalloc(s, &s->d_side, (size_t)s->m * sizeof(double2)));
        HIP_OK(launch_build_side(s->vk, s->rows, s->d_b64, s->d_side, s->st));
    }
    if (p.trace) {
        const int64_t waves = (R * G + 63) / 64;
        if (s->trace_cap < waves) {
            (void)hipFree(s->d_trace);
            s->d_trace = nullptr;
            s->trace_cap = 0;
            HIP_OK(hipMalloc((void **)&s->d_trace, (size_t)waves * kTraceWords * 8));
            s->trace_cap = waves;
        }
        if (!s->d_tau) {
            HIP_OK(hipMalloc((void **)&s->d_tau, (size_t)kTauShards * kTauShardStride * 8));
            HIP_OK(launch_zero(s->d_tau, (int64_t)kTauShards * kTauShardStride * 8, s->st));
        }
    }
    const bool monitor = p.tol > 0.0 || p.history_cap > 0 || p.cancel != nullptr;
    double err0 = NAN;
    auto push_hist = [&](double e) {
        if (S.history_len < p.history_cap) p.history[S.history_len++] = e;
    };
    const double t_setup = now_s();

    double gpu_s = 0.0;
    TraceSums tr;
    asyrk_status result = ASYRK_OK;
    int64_t ticket = p.ticket0;
    int64_t done = 0;

    if (!p.refine) {
        HIP_OK(launch_cast_to_iter(s->d_x64, s->d_x, f32, xsh, s->n, s->st));
        if (monitor) {
            asyrk_status rc = monitored_error(s, mon, s->d_x, f32, xsh, &err0);
            if (rc) return rc;
            push_hist(err0);
            S.final_err = err0;
            if (p.tol > 0.0 && err0 <= p.tol) sweeps = 0;
        }
        while (done < sweeps) {
            const int64_t c = std::min<int64_t>(p.check_every, sweeps - done);
            asyrk_status rc = run_sweeps(s, p, xk, G, R, gamma, seed, ticket, ticket + c * s->m, &gpu_s, &tr);
            if (rc) return rc;
            ticket += c * s->m;
            done += c;
            if (monitor || done == sweeps) {
                double e = 0.0;
                rc = monitored_error(s, mon, s->d_x, f32, xsh, &e);
                if (rc) return rc;
                S.final_err = e;
                push_hist(e);
                if (!std::isfinite(e) || (std::isfinite(err0) && err0 > 0 && e > 1e6 * err0)) {
                    result = ASYRK_ERR_DIVERGED;
                    break;
                }
                if (p.tol > 0.0 && e <= p.tol) break;
                if (p.cancel && *p.cancel) {
                    result = ASYRK_ERR_CANCELLED;
                    break;
                }
            }
        }
        // x is returned untouched when no sweep ran (no FP32 round trip)
        if (done > 0) HIP_OK(launch_iter_to_f64(s->d_x, f32, xsh, s->d_x64, s->n, 0, s->st));
        if (result == ASYRK_OK && p.tol > 0.0 && !(S.final_err <= p.tol)) result = ASYRK_ERR_NOT_CONVERGED;
    } else {
        // FP64 iterative refinement: x64 master, FP32 correction d on A d = fp32(b - A x64).
        // inner_sweeps > 0: that many sweeps per inner solve.  inner_sweeps = 0:
        // the inner solve stops when its own relative residual ||r32 - A d|| /
        // ||r32|| is <= 1e-6 or stops improving (the FP32 floor), at most 40.
        const bool adaptive = p.inner_sweeps == 0;
        const int64_t inner = adaptive ? 40 : p.inner_sweeps;
        asyrk_status rc = monitored_error(s, mon, s->d_x64, 0, 0, &err0);
        if (rc) return rc;
        push_hist(err0);
        S.final_err = err0;
        bool ok = p.tol > 0.0 && err0 <= p.tol;
        // Adaptive inner solves: the first one checks its residual after every
        // sweep; the later ones solve with the same matrix from d = 0 and
        // reach the FP32 floor in about as many sweeps, so they run that many
        // without checks (the outer FP64 error still decides convergence).
        int64_t learned = 0;
        while (!ok && done < sweeps) {
            // r = b - A x64 into the records' b fields (FP32), d = 0
            HIP_OK(launch_residual(s->vk, s->rows, s->d_b64, s->d_x64, 0, 0, nullptr, 1, s->d_part, kResidualBlocks,
                                   s->st));
            s->rec_b_dirty = true;
            HIP_OK(launch_zero(s->d_x, s->n * s->xstride, s->st));
            const int64_t budget = std::min<int64_t>(inner, sweeps - done);
            if (!adaptive) {
                rc = run_sweeps(s, p, xk, G, R, gamma, seed, ticket, ticket + budget * s->m, &gpu_s, &tr);
                if (rc) return rc;
                ticket += budget * s->m;
                done += budget;
            } else if (learned > 0) {
                const int64_t k = std::min(learned, budget);
                rc = run_sweeps(s, p, xk, G, R, gamma, seed, ticket, ticket + k * s->m, &gpu_s, &tr);
                if (rc) return rc;
                ticket += k * s->m;
                done += k;
            } else {
                double r0 = 0.0, prev = 1.0;
                HIP_OK(launch_residual(s->vk, s->rows, nullptr, s->d_x, 1, xsh, nullptr, 0, s->d_part, kResidualBlocks,
                                       s->st, 1));
                rc = fetch_scalar(s, kResidualBlocks, &r0);
                if (rc) return rc;
                for (int64_t k = 0; k < budget; ++k) {
                    rc = run_sweeps(s, p, xk, G, R, gamma, seed, ticket, ticket + s->m, &gpu_s, &tr);
                    if (rc) return rc;
                    ticket += s->m;
                    done += 1;
                    learned = k + 1;
                    double rk = 0.0;
                    HIP_OK(launch_residual(s->vk, s->rows, nullptr, s->d_x, 1, xsh, nullptr, 0, s->d_part,
                                           kResidualBlocks, s->st, 1));
                    rc = fetch_scalar(s, kResidualBlocks, &rk);
                    if (rc) return rc;
                    const double rel = r0 > 0 ? std::sqrt(rk / r0) : 0.0;
                    if (!std::isfinite(rel) || rel <= 1e-6 || rel > 0.5 * prev) break;
                    prev = rel;
                }
            }
            HIP_OK(launch_iter_to_f64(s->d_x, 1, xsh, s->d_x64, s->n, 1, s->st));
            S.outer_iters++;
            double e = 0.0;
            rc = monitored_error(s, mon, s->d_x64, 0, 0, &e);
            if (rc) return rc;
            S.final_err = e;
            push_hist(e);
            if (!std::isfinite(e) || (err0 > 0 && e > 1e6 * err0)) {
                result = ASYRK_ERR_DIVERGED;
                break;
            }
            if (p.tol > 0.0 && e <= p.tol) ok = true;
            if (p.cancel && *p.cancel) {
                result = ASYRK_ERR_CANCELLED;
                break;
            }
        }
        HIP_OK(launch_set_rec_b(s->vk, s->rows, s->d_b64, s->st));
        s->rec_b_dirty = false;
        if (result == ASYRK_OK && p.tol > 0.0 && !ok) result = ASYRK_ERR_NOT_CONVERGED;
    }
    // ||b - A x|| / ||b|| of the returned iterate: the monitor's last value when
    // it measured exactly that, else one FP64 residual pass
    S.final_resid = NAN;
    if (!p.skip_resid) {
        const bool have = !mon.use_ref && (p.refine || done > 0 || monitor);
        if (have) {
            S.final_resid = S.final_err;
        } else {
            if (mon.use_ref) {
                HIP_OK(launch_sumsq_diff(s->d_b64, 0, 0, nullptr, s->m, s->d_part, kResidualBlocks, s->st));
                asyrk_status rc = fetch_scalar(s, kResidualBlocks, &mon.b_norm2);
                if (rc) return rc;
            }
            double v = 0.0;
            HIP_OK(launch_residual(s->vk, s->rows, s->d_b64, s->d_x64, 0, 0, nullptr, 0, s->d_part, kResidualBlocks,
                                   s->st));
            asyrk_status rc = fetch_scalar(s, kResidualBlocks, &v);
            if (rc) return rc;
            S.final_resid = mon.b_norm2 > 0 ? std::sqrt(v / mon.b_norm2) : std::sqrt(v);
        }
    }
    HIP_OK(hipMemcpyAsync(x, s->d_x64, (size_t)s->n * 8, d2h, s->st));
    HIP_OK(hipStreamSynchronize(s->st));

    S.sweeps_done = done;
    S.row_updates = done * s->m;
    S.next_ticket = ticket;
    S.seconds = now_s() - t_setup;
    (void)wall0;
    S.sweep_seconds = gpu_s;
    S.rows_per_s = gpu_s > 0 ? (double)S.row_updates / gpu_s : 0.0;
    if (p.trace && tr.count > 0) {
        int clock_khz = 0;
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev);
        const double ns_per_tick = clock_khz > 0 ? 1e6 / clock_khz : 10.0;
        S.tau_samples = (int64_t)tr.count;
        S.tau_obs_mean = tr.tau_sum / tr.count;
        S.tau_obs_max = tr.tau_max;
        S.window_ns_mean = tr.win_sum / tr.count * ns_per_tick;
        S.window_ns_max = tr.win_max * ns_per_tick;
    }
    // Corollary 1's bound on tau for this system
    S.lambda_source = s->lambda_pi > 0.0 ? 1 : 0;
    S.lambda_max_est = S.lambda_source ? s->lambda_pi : std::max(lambda_mp(s), s->max_col_norm2);
    const double tmax = std::floor(s->fro2 / (2.0 * M_E * S.lambda_max_est)) - 1.0;
    S.tau_max_corollary = tmax >= 0.0 ? tmax : -1.0;
    if (st) *st = S;
    return result;
}

}  // extern "C"
