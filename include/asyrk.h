/*
 * asyrk.h - C ABI of the MI355X (gfx950) asynchronous randomized Kaczmarz
 * library.
 *
 * The method (Liu, Wright, Sridhar, "An Asynchronous Parallel Randomized
 * Kaczmarz Algorithm"): solve a consistent sparse system A x = b, A (m x n)
 * with no zero rows (Section 1, eq. (1)).  Many workers run concurrently over
 * one shared iterate x; each one repeatedly
 *   1. draws row i with probability ||a_i||^2 / ||A||_F^2 (Section 1),
 *   2. reads x on supp(a_i) without locking, possibly stale (Section 3),
 *   3. forms r = a_i^T x - b_i,
 *   4. writes x <- x - gamma * r / ||a_i||^2 * a_i on every coordinate of
 *      supp(a_i) with lock-free atomic additions (eq. (2) with a step length
 *      gamma; the all-coordinate variant of Section "Experiments", which on
 *      one worker is plain randomized Kaczmarz).
 * The delay between a worker's read and its write is the tau of eq. (3);
 * Corollary 1 bounds the number of workers for near-linear speedup by
 * 2 e lambda_max (tau + 1) / m <= 1.
 *
 * Conventions for every call
 *   - Every call returns an asyrk_status; none aborts, throws or exits.
 *   - Pointer arguments are host pointers or device pointers as selected by
 *     the `mem` argument of asyrk_create (ASYRK_MEM_HOST / ASYRK_MEM_DEVICE);
 *     that choice holds for every later call on the same system.  Exception:
 *     structs (params, stats, info) and scalar outputs are always host memory.
 *   - The caller owns every array it passes.  asyrk_create copies what it
 *     needs; nothing passed in is retained after a call returns.
 *   - All GPU work of a system is enqueued on the HIP stream given to
 *     asyrk_create (NULL = the null stream) and every call synchronizes that
 *     stream before it returns.
 *   - One host thread at a time per system; separate systems are independent.
 *   - Row indices are int32: m, n < 2^31 and each row has < 2^31 entries.
 *
 * Device layout (owned by the system): each row is one packed record of a
 * 16-byte header (b_i, 1/||a_i||^2, alias threshold, alias row; 32 bytes for
 * FP64) followed by its (column, value) pairs in groups of 4 (8 for BF16),
 * padded to 16 or 64 bytes.  Equal-length rows sit at a fixed stride; other
 * systems keep an 8-byte (offset, length) entry per row.
 */
#ifndef ASYRK_H
#define ASYRK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASYRK_ABI_VERSION 3

typedef struct asyrk_system asyrk_system; /* opaque; owns all device-side data */

typedef enum asyrk_status {
    ASYRK_OK = 0,
    ASYRK_ERR_INVALID_ARG = 1,   /* an argument fails validation (nothing was changed) */
    ASYRK_ERR_ZERO_ROW = 2,      /* a row of A has ||a_i|| = 0 (Section 1 excludes it) */
    ASYRK_ERR_OOM = 3,           /* device or host allocation failed */
    ASYRK_ERR_DEVICE = 4,        /* a HIP runtime call failed (no GPU, launch error) */
    ASYRK_ERR_NOT_CONVERGED = 5, /* tol > 0 and the sweep budget ran out; x and stats are valid */
    ASYRK_ERR_DIVERGED = 6,      /* the monitored error became non-finite or grew 1e6-fold */
    ASYRK_ERR_CANCELLED = 7,     /* the cancel flag was set; x holds the last checked iterate */
    ASYRK_ERR_UNSUPPORTED = 8,   /* a valid combination this build does not implement */
    ASYRK_PENDING = 9,           /* asyrk_server_poll: the request has not finished yet */
    ASYRK_ERR_SCRATCH = 10       /* the problem does not fit the fixed scratch of an
                                    allocation-free entry point (nothing was changed) */
} asyrk_status;

typedef enum asyrk_dtype { ASYRK_F64 = 0, ASYRK_F32 = 1, ASYRK_BF16 = 2 } asyrk_dtype;
typedef enum asyrk_mem { ASYRK_MEM_HOST = 0, ASYRK_MEM_DEVICE = 1 } asyrk_mem;

/* ASYNC: many workers, lock-free (Section 3).  REPLAY: one worker, tickets
 * strictly in order, deterministic: plain randomized Kaczmarz (eq. (2)). */
typedef enum asyrk_mode { ASYRK_ASYNC = 0, ASYRK_REPLAY = 1 } asyrk_mode;

/* NORM2: P(i) = ||a_i||^2/||A||_F^2 (Section 1).  UNIFORM: P(i) = 1/m
 * (Algorithm 1's equal probability; the same thing for normalized rows). */
typedef enum asyrk_sampling { ASYRK_SAMPLE_NORM2 = 0, ASYRK_SAMPLE_UNIFORM = 1 } asyrk_sampling;

/* ALL: every coordinate of supp(a_i) (eq. (2), Section "Experiments").
 * ONE: one coordinate t uniform in supp(a_i), step gamma*theta_i
 * (Algorithm 1, the variant Theorem 1 and Corollary 1 analyse). */
typedef enum asyrk_update { ASYRK_UPDATE_ALL = 0, ASYRK_UPDATE_ONE = 1 } asyrk_update;

/* Random row selection for ticket j (identical on every device and in every
 * mode, so REPLAY is reproducible and resumable):
 *   (u0,u1,u2,u3) = Philox4x32-10(counter = (j mod 2^32, j div 2^32, stream_id, 0),
 *                                 key = (seed mod 2^32, seed div 2^32))
 *   k = floor((u1 * 2^32 + u0) * m / 2^64)
 *   NORM2:   i = (u2 < T_k) ? k : alias_k, with (T, alias) the Vose alias table
 *            of the row weights ||a_i||^2 (T_k in [0, 2^32])
 *   UNIFORM: i = k
 *   UPDATE_ONE: t = floor(u3 * theta_i / 2^32), the position inside row i. */

typedef struct asyrk_solve_params {
    int32_t mode;            /* asyrk_mode, default ASYNC */
    int32_t sampling;        /* asyrk_sampling, default NORM2 */
    int32_t update;          /* asyrk_update, default ALL */
    int32_t lanes;           /* lanes per row G in {1,2,4,8,16,32,64}; 0 = the autotuned
                                value when the autotuner ran at this R, else the largest
                                power of two with R * G <= 65536, capped by the smallest
                                power of two covering the longest row's units (and 64) */
    int64_t in_flight;       /* R, row workers in flight (tau_design = R - 1); 0 = choose */
    double tol;              /* stop when the monitored error <= tol; 0 = run every sweep */
    const double *x_ref;     /* nullable, length n: monitor ||x - x_ref||/||x_ref||;
                                when NULL the monitor is ||A x - b||/||b|| */
    int32_t check_every;     /* sweeps between error checks (>= 1), default 1 */
    int32_t refine;          /* 1: FP64 iterative refinement around FP32 sweeps (see asyrk_solve) */
    int64_t inner_sweeps;    /* refinement: sweeps per inner solve, 0 = choose: the first inner
                                solve stops when its relative residual is <= 1e-6 or stops
                                halving per sweep (at most 40), later ones run as many sweeps */
    uint32_t stream_id;      /* RNG stream (third counter word) */
    int32_t trace;           /* 1: measure the staleness of eq. (3) in every sweep kernel and
                                worker loop (see asyrk_solve_stats.tau_obs_mean): a completion
                                counter that each wave advances once per step, read by every
                                wave on one step in 16 just before its gathers and right
                                after its scatter */
    int64_t ticket0;         /* first ticket (resume: pass stats.next_ticket) */
    volatile const int32_t *cancel; /* nullable HOST pointer, polled at every check */
    double *history;         /* nullable HOST array: monitored error at the start and after
                                each check (refinement: after each outer iteration) */
    int64_t history_cap;     /* capacity of history */
    int32_t iter_dtype;      /* iterate and sweep arithmetic: -1 (set by
                                asyrk_solve_params_init) = ASYRK_F64, or ASYRK_F32 with
                                refine = 1; ASYRK_F32 (F32/BF16 values only: FP32
                                atomics) or ASYRK_F64 (any values; FP64 atomics, which
                                this GPU executes faster than FP32 ones; FP32/BF16 values
                                then take b_i and 1/||a_i||^2 in FP64 from side records
                                of 16 bytes per row, built on first use) */
    int32_t order;           /* 0: each ticket draws its row (with replacement, default);
                                1: the paper's experimental scheme: worker w owns rows
                                [w L, (w+1) L), L = ceil(m / R), and visits each of
                                them once per sweep in a keyed permutation (see
                                "Slice permutation"); needs UPDATE_ALL and ticket0 a
                                multiple of m */
    int32_t pipeline;        /* worker loop: 1 = pipelined (each worker fetches its next
                                ticket's row while the current one gathers and scatters:
                                same arithmetic and reads of x, two dependent memory
                                round trips per ticket; faster when few workers are in
                                flight, slower when the atomic unit is saturated);
                                2 = batched (each worker fetches the rows of its next
                                8, 4 or 2 tickets together, for G >= 8, G = 4 and
                                G <= 2, and runs them back to back: same arithmetic and
                                reads of x, one record round trip per batch; the
                                fastest loop with few workers in flight; with G = 64
                                and R <= 512 each worker is two waves of one
                                workgroup, one fetching the next batch's records into
                                LDS while the other computes).  1 and 2 need
                                ASYNC and UPDATE_ALL (with order 1 each worker's slice
                                walk is its ticket stream).  0 = plain.
                                -1 (set by asyrk_solve_params_init) = the autotuned
                                choice when the autotuner ran at this R and G, else
                                batched for R <= 1024 and pipelined for R <= 8192
                                where allowed */
    int32_t skip_resid;      /* 0 (default): fill asyrk_solve_stats.final_resid, which costs one
                                FP64 residual pass unless the monitor already measured the
                                residual of the returned x; 1: leave it NaN */
} asyrk_solve_params;

/* Slice permutation (order = 1), for sweep s (= ticket / m) and worker w:
 *   (u0,u1,u2,u3) = Philox4x32-10(counter = (s mod 2^32, s div 2^32, w, 0x5C4E3D2B), key = seed)
 *   position k of the worker's L_w rows maps to start_w + P(k), where P walks
 *   y = k through  y <- ((y ^ (y >> h)) * (u0 | 1) + u1) & mask,
 *                  y <- ((y ^ (y >> h)) * (u2 | 1) + u3) & mask
 *   (32-bit arithmetic; b = smallest width with 2^b >= L_w, mask = 2^b - 1,
 *   h = (b + 1) / 2) until y < L_w.  REPLAY (one worker) visits all m rows in
 *   that order each sweep. */

typedef struct asyrk_solve_stats {
    int64_t sweeps_done;       /* sweeps (m tickets each) performed */
    int64_t row_updates;       /* tickets performed */
    int64_t next_ticket;       /* ticket0 + row_updates */
    int64_t history_len;       /* entries written to params.history */
    int64_t in_flight;         /* R used */
    int32_t lanes;             /* G used */
    int32_t outer_iters;       /* refinement outer iterations (0 without refinement) */
    int32_t pipelined;         /* worker loop that ran: 0 plain, 1 pipelined, 2 batched */
    int32_t reserved;
    double seconds;            /* wall time of the call after setup */
    double sweep_seconds;      /* GPU time of the sweep kernels (HIP events) */
    double rows_per_s;         /* row_updates / sweep_seconds */
    double final_err;          /* last monitored error (NaN if never checked) */
    double tau_design;         /* R - 1 */
    double tau_obs_mean;       /* trace: eq. (3)'s delay j - k(j) measured on sampled tickets: the
                                  row updates other workers completed between the ticket's read
                                  of x and its scatter (completion counter, advanced once per
                                  wave and step after the scatter is issued); mean over samples */
    double tau_obs_max;        /* trace: the largest sampled delay */
    double window_ns_mean;     /* trace: mean time from the sampled read to the scatter, ns */
    double window_ns_max;      /* trace: its maximum, ns */
    int64_t tau_samples;       /* trace: number of sampled (wave, step) pairs */
    double lambda_max_est;     /* lambda_max(A^T A) behind tau_max_corollary: the power-iteration
                                  value once asyrk_lambda_max has run on this system, else
                                  max(Gaussian-ensemble estimate, largest column norm^2) */
    double tau_max_corollary;  /* Corollary 1: the largest tau with
                                  2 e lambda_max_est (tau + 1) / ||A||_F^2 <= 1, or -1 if none */
    double final_resid;        /* ||b - A x|| / ||b|| of the returned x in FP64 (the quantity of the
                                  paper's figures, Section "Experiments"); NaN with skip_resid */
    int32_t lambda_source;     /* 1: lambda_max_est is a power-iteration value; 0: the estimate */
    int32_t reserved2;
} asyrk_solve_stats;

typedef struct asyrk_system_info {
    int64_t m, n, nnz;
    int64_t mu;                /* max_i ||a_i||_0 (Section 1 notation) */
    int64_t nu;                /* max_j ||column j||_0 */
    int64_t fixed_nnz;         /* common row length, or 0 if rows differ */
    int64_t record_stride;     /* bytes per row record when fixed_nnz > 0 */
    int64_t device_bytes;      /* device memory held by the system */
    int32_t vals_dtype;        /* asyrk_dtype of the stored values */
    int32_t iter_dtype;        /* default iterate dtype (ASYRK_F64) */
    double fro2;               /* ||A||_F^2 (FP64, stored values) */
    double lambda_mp;          /* (1 + sqrt(n/m))^2 * fro2 / n: Gaussian-ensemble estimate of lambda_max */
    int64_t record_bytes_per_row; /* algorithmic bytes per row update (values, indices, b_i, w_i, start) */
    double max_col_norm2;      /* max_j ||column j||^2, a lower bound on lambda_max */
    int64_t default_in_flight; /* R used when in_flight = 0: Corollary 1's bound with
                                  lambda = max(lambda_mp, max_col_norm2), in [1, 65536] */
    int64_t iterate_stride;    /* bytes between consecutive elements of the device-side sweep
                                  iterate: 256 for n <= 2^20, 64 for n <= 2^23, else 8.
                                  Columns sharing a cache line make their gathers and atomics
                                  queue behind each other; the caller's x stays dense */
    int64_t tuned_in_flight;   /* R chosen by asyrk_autotune(in_flight = -1) for the FP64
                                  iterate, used by solves with in_flight = 0; 0 if none */
} asyrk_system_info;

/* Version of this ABI (ASYRK_ABI_VERSION). */
int asyrk_abi_version(void);

/* Static string for a status code. */
const char *asyrk_status_string(asyrk_status s);

/* Text of the last HIP runtime error seen by this thread ("" if none). */
const char *asyrk_last_error_message(void);

/* Default parameters (ASYNC, NORM2, ALL, G and R chosen, check every sweep). */
void asyrk_solve_params_init(asyrk_solve_params *p);

/*
 * Build a system from CSR A and b (Section 1, eq. (1)).
 *   row_ptr  int64[m+1], row_ptr[0] = 0, non-decreasing
 *   col_idx  int32[nnz], 0 <= c < n, strictly increasing inside each row
 *   vals     nnz values of type vals_dtype (F64, F32, or BF16 bit patterns);
 *            these stored values ARE the matrix: FP64 work promotes them exactly
 *   b        double[m], finite
 *   mem      ASYRK_MEM_HOST or ASYRK_MEM_DEVICE for every pointer argument
 *   stream   hipStream_t (as void *), NULL for the null stream
 * Sweeps run in FP64 (values F64) or, by default, FP32 (values F32/BF16);
 * asyrk_solve_params.iter_dtype = ASYRK_F64 runs FP32/BF16 values with an
 * FP64 iterate and FP64 atomics.
 * With ASYRK_MEM_DEVICE only row_ptr and the row weights pass through host
 * memory: the entries are validated, weighed and packed into the row records
 * on the device, from the caller's arrays (which are read during the call
 * only), with the same records, statuses and statistics as host inputs give
 * (max_col_norm2 up to the rounding order of its sums).
 * Errors: INVALID_ARG (shape, ordering, range, non-finite), ZERO_ROW, OOM,
 * DEVICE.  On error *out is set to NULL.
 */
asyrk_status asyrk_create(asyrk_system **out, int64_t m, int64_t n, const int64_t *row_ptr,
                          const int32_t *col_idx, const void *vals, int32_t vals_dtype,
                          const double *b, int32_t mem, void *stream);

/*
 * Least squares for an inconsistent A x = b through the consistent augmented
 * system of the paper's Section "Extension to Inconsistent Systems":
 *     [ 0      phi A^T ] [x]   [phi A^T b]
 *     [ A     -zeta I  ] [y] = [    0    ]
 * (size n + m; zeta, phi > 0; the paper's best choice is phi = 1 and
 * zeta = sigma_min(A) / sqrt(2)).  Arguments as in asyrk_create for A and b;
 * the created system's unknown is z = (x, y) and its x block equals
 * zeta * x_LS; asyrk_augmented_solution returns x_LS = z[0:n] / zeta.  Entries
 * phi * a_ij and -zeta are rounded to vals_dtype.  Errors as asyrk_create;
 * ZERO_ROW also for an empty column of A.
 */
asyrk_status asyrk_create_augmented(asyrk_system **out, int64_t m, int64_t n, const int64_t *row_ptr,
                                    const int32_t *col_idx, const void *vals, int32_t vals_dtype,
                                    const double *b, double zeta, double phi, int32_t mem, void *stream);

/*
 * The least-squares solution of a system made by asyrk_create_augmented, from
 * the augmented unknown z = (x, y) (double[n + m], e.g. asyrk_solve's result):
 * x_out[k] = z[k] / zeta for k < n (Section "Extension to Inconsistent
 * Systems": the x block of the augmented solution is zeta x_LS).  z and x_out
 * (double[n], n of the original A) are in the system's memory kind and may
 * alias.  Errors: INVALID_ARG (s not augmented, NULL pointers), DEVICE.
 */
asyrk_status asyrk_augmented_solution(asyrk_system *s, const double *z, double *x_out);

/* Release every device and host resource of the system (NULL is accepted). */
asyrk_status asyrk_destroy(asyrk_system *s);

/* Replace b (double[m], finite; in the memory kind the system was created
 * with, read during the call only) keeping A.  Device b is checked on the
 * device.  INVALID_ARG for a non-finite entry, with the system's b unchanged. */
asyrk_status asyrk_set_rhs(asyrk_system *s, const double *b);

/* Sizes and derived quantities of the system. */
asyrk_status asyrk_system_info_get(const asyrk_system *s, asyrk_system_info *info);

/*
 * Copy of the packed row records (headers {b_i, 1/w_i, alias bucket}, the
 * rows' (column, value) units and their padding, laid out as the sweep reads
 * them) into host memory dst of cap bytes, for checking the setup; the
 * headers carry the current b.  *bytes_out (nullable) receives the image's
 * size; dst = NULL only queries it.  INVALID_ARG for s = NULL or cap below
 * the size.  Synchronizes the system's stream.
 */
asyrk_status asyrk_records_get(asyrk_system *s, void *dst, int64_t cap, int64_t *bytes_out);

/*
 * Run the method from x (double[n], in: x0, out: the final iterate).
 *   gamma   step length, 0 < gamma < 2 (eq. (2) scaled; gamma = 1 is the
 *           orthogonal projection)
 *   sweeps  budget in sweeps of m tickets: tickets ticket0 .. ticket0 + sweeps*m - 1
 *   seed    Philox key
 *   p       NULL for defaults (asyrk_solve_params_init)
 *   st      nullable; filled on OK, NOT_CONVERGED, DIVERGED and CANCELLED
 * ASYNC runs R workers at once; staleness is not bounded by construction
 * (tau_design = R - 1 is the modeling value; trace measures windows).
 * REPLAY forces one worker and is bitwise reproducible.
 * With refine = 1 (FP32 iterate only): outer loop r = b - A x in FP64,
 * inner sweeps on A d = fp32(r) from d = 0, x += d in FP64, until the
 * monitored error <= tol or the budget is spent.  The system's b is
 * restored before return.
 * Errors: INVALID_ARG, DEVICE, NOT_CONVERGED, DIVERGED, CANCELLED.
 */
asyrk_status asyrk_solve(asyrk_system *s, double *x, double gamma, int64_t sweeps,
                         uint64_t seed, const asyrk_solve_params *p, asyrk_solve_stats *st);

/*
 * Residual in FP64 over the stored values promoted exactly:
 *   r = b - A x (x double[n]); r_out nullable double[m]; *norm2_out = ||r||^2,
 * the squared residual norm the paper plots against epochs (Section
 * "Experiments").  x and r_out are in the system's memory kind.
 * Errors: INVALID_ARG, DEVICE.
 */
asyrk_status asyrk_residual(asyrk_system *s, const double *x, double *r_out, double *norm2_out);

/*
 * Rows the device sampler draws for tickets ticket0 .. ticket0+count-1
 * (see "Random row selection" above); rows_out int32[count].  With
 * coords_out (nullable int32[count]) also the position t used by UPDATE_ONE.
 */
asyrk_status asyrk_sample_rows(asyrk_system *s, uint64_t seed, uint32_t stream_id, int32_t sampling,
                               int64_t ticket0, int64_t count, int32_t *rows_out,
                               int32_t *coords_out);

/*
 * lambda_max(A^T A) (Section 1 notation) by power iteration on the GPU,
 * from a Philox-seeded start; *lambda_out gets the Rayleigh quotient after
 * iters steps (iters >= 1).  tau_max_out (nullable): the largest tau with
 * 2 e lambda_max (tau + 1) / ||A||_F^2 <= 1 (Corollary 1; ||A||_F^2 = m for
 * normalized rows), or -1 when none.  The system keeps the value for the
 * lambda_max_est and tau_max_corollary of later solves.
 */
asyrk_status asyrk_lambda_max(asyrk_system *s, int32_t iters, uint64_t seed, double *lambda_out,
                              double *tau_max_out);

/*
 * asyrk_lambda_max without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid it): the same power iteration and the same outputs, with its
 * vectors v, z (n doubles each), y (m doubles) and reduction partials in one
 * fixed 64 MiB device array that the library holds on every device it runs
 * on until the process ends.  Calls no hipMalloc, hipFree or allocating
 * library routine; the result reaches the host through the system's pinned
 * scalar.  Requires 2 n + m + 2049 <= 8,388,608 (doubles) and the system's
 * device current.  Every call on one device shares that array: calls that
 * overlap on one GPU (several host threads, or streams running concurrently)
 * race and must be serialized by the caller.
 * Errors: INVALID_ARG (NULL, iters < 1, another device current), SCRATCH (too
 * large; asyrk_last_error_message says so), DEVICE.
 */
asyrk_status asyrk_lambda_max_noalloc(asyrk_system *s, int32_t iters, uint64_t seed, double *lambda_out,
                                      double *tau_max_out);

/*
 * Autotuner: times one sweep (at least 2^21 tickets) from x = 0 for each
 * lane-group width G in {1, 2, 4, 8, 16, 32, 64} and each worker loop (plain,
 * pipelined, batched) on this system, at in_flight workers (0 = the default R) and the
 * given iterate dtype (-1 = default), and keeps the fastest pair for later
 * solves with lanes = 0 and pipeline = -1 at that R.  in_flight = -1 chooses R
 * as well: each power of two from 1024 below the default R, and the default R,
 * is timed with its best pair, and the smallest R within 2% of the fastest is
 * kept (the same throughput with less staleness); later asynchronous,
 * all-coordinate solves with replacement and in_flight = 0 then use it
 * (asyrk_system_info.tuned_in_flight); other kinds keep the default R.  Near-ties go by a fixed
 * rule: a loop replaces the one chosen so far (plain, then pipelined, then
 * batched) only when its best rate is more than 3% higher, then the smallest G
 * within 3% of that loop's best.  best_lanes and best_pipeline (nullable)
 * receive it; rows_per_s (nullable, double[21]) the rate of each candidate:
 * [0..6] plain, [7..13] pipelined, [14..20] batched, G ascending.  The
 * system's b and matrix are unchanged.  Errors: INVALID_ARG, UNSUPPORTED,
 * DEVICE.
 */
asyrk_status asyrk_autotune(asyrk_system *s, double gamma, int32_t iter_dtype, int64_t in_flight,
                            int32_t *best_lanes, int32_t *best_pipeline, double *rows_per_s);

/*
 * Device ceilings used to read the roofline (no system needed):
 *   asyrk_probe_copy      streaming copy of `bytes` bytes, `iters` times;
 *                         *gbps = 2*bytes*iters / time (read + write)
 *   asyrk_probe_scatter   `count` random 4- or 8-byte accesses (kind 0:
 *                         agent-coherent loads, 1: atomic add) over a
 *                         table of `n` elements of dtype F32 or F64;
 *                         *per_s = accesses per second
 * Errors: INVALID_ARG, OOM, DEVICE.
 */
asyrk_status asyrk_probe_copy(int64_t bytes, int32_t iters, double *gbps);
asyrk_status asyrk_probe_scatter(int64_t n, int64_t count, int32_t dtype, int32_t kind,
                                 int32_t iters, double *per_s);

/* ------------------------------------------------------------------------
 * Serving: many independent systems with continuous batching.
 *
 * Each request is a consistent system with FP32 values, solved to
 * ||b - A x|| <= tol ||b|| by asynchronous sweeps (row workers bounded by the
 * system's own Corollary 1 limit; FP64 correction and FP64 atomics over the
 * FP32 values) inside an FP64 refinement loop (r = b - A x, d from A d = r,
 * x += d).  The active systems form two groups whose rounds alternate on
 * two streams; one progress() call collects one group's previous round
 * (retiring finished requests), lets uploaded requests join it, admits
 * queued requests (uploads on a copy stream) and launches the group's next
 * round, one packed launch per phase over its systems, while the other
 * group's round computes.  Requests that arrive meanwhile are admitted as
 * slots, workers and device memory free up.  A request's result does not depend on what else is in the batch
 * beyond the nondeterminism of asynchronous execution.
 * Threads: submit/poll/stats may be called from any thread; progress from one
 * thread at a time.
 * ------------------------------------------------------------------------ */
typedef struct asyrk_server asyrk_server;

typedef struct asyrk_server_config {
    int64_t budget_bytes;  /* device memory for resident systems (one arena), default 64 GiB */
    int32_t max_slots;     /* systems active at once in each round group, default 1024 */
    int32_t inner_sweeps;  /* sweeps per round (refinement inner solve), default 8; a request's
                              later rounds may run fewer (see fixed_rounds) */
    int64_t max_workers;   /* row workers of one group's round, default 65536 (both groups
                              together: 1.5 times that; admitted, uploading: twice that) */
    int32_t max_rounds;    /* per request; then NOT_CONVERGED, default 60 */
    int32_t use_graph;     /* 1: the round runs as one captured hipGraph, default 1 */
    double gamma;          /* step length in (0, 2), default 1 */
    int64_t pinned_bytes;  /* pinned host staging for queued requests (uploads become one DMA
                              each), default 4 GiB; 0 = none; a request that does not fit is
                              uploaded from pageable memory */
    int32_t lanes;         /* lanes per row in the packed sweep of busy rounds: 4 or 8 (each
                              keeps rows of up to 64 entries in registers), default 4; 0 =
                              tune online, per load bucket (active workers in [w, 2w) for
                              w = pipe_workers, 2 pipe_workers, 4 pipe_workers, and beyond):
                              a bucket's first rounds sweep their systems once per candidate
                              (4, 8; each twice, each first once), timed, the round's own
                              sweep last, and the fastest total is kept for the bucket */
    int32_t pipe_workers;  /* rounds whose active systems hold at most this many row workers
                              run the pipelined worker loop (see asyrk_solve_params.pipeline),
                              default 8192; 0 = never */
    int32_t pipe_lanes;    /* lanes per row in those rounds: 4, 8, 16 or 32, default 16 (fewer
                              entries per lane shorten each latency-bound ticket); 0 = tune
                              online among 4, 8, 16, 32 as for lanes, with the buckets below
                              pipe_workers / 4, below pipe_workers / 2, below pipe_workers,
                              and pipe_workers */
    int32_t fixed_rounds;  /* 0 (default): after each round a request's next round runs the
                              sweeps its measured contraction per sweep predicts it still needs
                              to reach tol, plus one, at most inner_sweeps; 1: always
                              inner_sweeps */
    int32_t order;         /* row order of every round: 1 (default) without replacement, the
                              slice scheme of asyrk_solve_params.order = 1 per system (worker w
                              of R_s owns rows [w L, (w+1) L), L = ceil(m / R_s), visited in a
                              fresh keyed permutation each sweep: fewer sweeps to tol), in busy
                              and pipelined rounds alike; 0: rows drawn with replacement */
    int32_t pinned_wait_ms; /* a submit whose packed request does not fit the pinned staging waits
                              up to this long for uploads to release some (default 1000; 0 =
                              never): admissions stay DMA transfers under overload instead of
                              pageable copies that hold the round loop's thread.  A caller that
                              also drives progress() itself from the submitting thread should
                              set 0 or keep the pinned staging large enough */
} asyrk_server_config;

typedef struct asyrk_request_stats {
    int64_t m, n, nnz;
    int64_t in_flight;     /* R_s */
    int64_t sweeps;        /* sweeps run (inner solves) */
    int32_t rounds;        /* refinement rounds */
    int32_t status;        /* ASYRK_OK, ASYRK_ERR_NOT_CONVERGED or ASYRK_ERR_DIVERGED */
    double rel_residual;   /* ||b - A x|| / ||b|| of the returned x (FP64) */
    double t_submit, t_admit, t_done;  /* asyrk_now() clock, seconds */
} asyrk_request_stats;

typedef struct asyrk_server_stats {
    int64_t submitted, admitted, completed, active, queued, rounds, row_updates, arena_used;
                           /* active: admitted and not finished (uploading, ready or in a group) */
    double gpu_seconds;    /* time the GPU spent in rounds: the union of the rounds' intervals
                              on the two group streams (HIP events) */
    int64_t round_workers;     /* row workers summed over rounds (/ rounds = mean per round) */
    int64_t round_systems;     /* active systems summed over rounds */
    int64_t pipelined_rounds;  /* rounds that ran the pipelined worker loop */
    int32_t lanes;             /* lanes per row of the last plain round's sweep */
    int32_t pipe_lanes;        /* lanes per row of the last pipelined round's sweep */
    int32_t lanes_tuning;      /* bit 0 / bit 1: the last plain / pipelined round timed every
                                  candidate width (its load bucket was still being tuned) */
    int32_t buckets_untuned;   /* load buckets (4 per loop) not tuned yet; 0 with fixed widths */
    int64_t pageable_uploads;  /* requests staged in pageable memory (no room in the pinned staging) */
} asyrk_server_stats;

/* Defaults for asyrk_server_config. */
void asyrk_server_config_init(asyrk_server_config *c);

/* Create a server (non-blocking HIP streams of its own: one per round group and
 * one for uploads; allocates the arena).
 * Errors: INVALID_ARG, OOM, DEVICE. */
asyrk_status asyrk_server_create(asyrk_server **out, const asyrk_server_config *cfg);

/* Destroy a server and every request it holds (NULL is accepted). */
asyrk_status asyrk_server_destroy(asyrk_server *s);

/* Queue one request: HOST arrays (CSR as in asyrk_create, FP32 values, FP64
 * b), tol > 0 on ||b - A x||/||b||, Philox seed.  The arrays are copied
 * (packed on the calling thread); *request_id receives its id.
 * Errors: INVALID_ARG, ZERO_ROW, OOM (larger than the whole budget), or the
 * server's sticky device failure. */
asyrk_status asyrk_server_submit(asyrk_server *s, int64_t m, int64_t n, const int64_t *row_ptr,
                                 const int32_t *col_idx, const float *vals, const double *b, double tol,
                                 uint64_t seed, int64_t *request_id);

/* Serve one round group: collect its previous round and retire finished
 * requests, add uploaded requests, admit what fits, launch its next round
 * (returns without waiting for it).  n_active / n_queued (nullable) receive
 * the counts afterwards.  Errors: DEVICE (or OOM) from a HIP call; such a
 * failure is sticky: this and every later progress and submit call, and poll
 * of every request not finished before it, return it (finished results stay
 * readable; destroy the server). */
asyrk_status asyrk_server_progress(asyrk_server *s, int32_t *n_active, int32_t *n_queued);

/* The round loop on the calling thread: progress() until *stop becomes
 * nonzero (the caller owns the flag and sets it from another thread); while
 * nothing is active or queued it sleeps until a submit, waking at least
 * every millisecond to read the flag.  Only one thread may run rounds on a
 * server at a time.  Errors: INVALID_ARG, or progress()'s DEVICE, which ends
 * the loop. */
asyrk_status asyrk_server_run(asyrk_server *s, const volatile int32_t *stop);

/* Result of a finished request: x_out (nullable, HOST double[n]) and stats
 * (nullable).  Returns the request's final status, ASYRK_PENDING while it is
 * queued or active, INVALID_ARG for an unknown or already-polled id, and the
 * server's sticky device failure for a request it left unfinished. */
asyrk_status asyrk_server_poll(asyrk_server *s, int64_t request_id, double *x_out,
                               asyrk_request_stats *st);

/* Ids of requests that finished since the last call (up to cap, oldest
 * first); *count receives how many were written.  Each id is reported once;
 * fetch its result with asyrk_server_poll.  Errors: INVALID_ARG. */
asyrk_status asyrk_server_take_completed(asyrk_server *s, int64_t *ids, int64_t cap, int64_t *count);

/* Counters of the server. */
asyrk_status asyrk_server_stats_get(asyrk_server *s, asyrk_server_stats *out);

/* The host clock the server's timestamps use (steady clock, seconds). */
double asyrk_now(void);

#ifdef __cplusplus
}
#endif

#endif /* ASYRK_H */
