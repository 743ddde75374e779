"""MI355X (gfx950) asynchronous randomized Kaczmarz: Python binding.

A thin ctypes layer over ``libasyrk.so`` (C ABI in ``include/asyrk.h``): it
marshals arguments and nothing else; every step of the method runs in the
library's HIP kernels.  Arrays are either all numpy (host memory) or all torch
CUDA tensors (device memory, work enqueued on torch's current stream).

    from paper_1401_4780_amd import System
    s = System(row_ptr, col, val, b)            # CSR A, right-hand side b
    st = s.solve(x, gamma=1.0, sweeps=30, seed=1, tol=1e-6, x_ref=x_star)

The library must be built first (``python -m paper_1401_4780_amd.build``);
importing works without it, but any call raises ``LibraryMissing``.
"""
from __future__ import annotations

import ctypes as C
import math
from pathlib import Path

import numpy as np

__all__ = ["System", "Server", "AsyrkError", "LibraryMissing", "lib", "library_path", "probe_copy",
           "probe_scatter", "now", "STATUS", "F64", "F32", "BF16"]

LIB_PATH = Path(__file__).resolve().parent / "_build" / "libasyrk.so"

F64, F32, BF16 = 0, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
ASYNC, REPLAY = 0, 1
SAMPLE_NORM2, SAMPLE_UNIFORM = 0, 1
UPDATE_ALL, UPDATE_ONE = 0, 1
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "ZERO_ROW", 3: "OOM", 4: "DEVICE", 5: "NOT_CONVERGED",
          6: "DIVERGED", 7: "CANCELLED", 8: "UNSUPPORTED", 9: "PENDING", 10: "SCRATCH"}
_SOFT = {5, 6, 7}  # statuses after which x and the stats are still valid


class LibraryMissing(RuntimeError):
    pass


class AsyrkError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{where}: {self.name}" + (f" ({detail})" if detail else ""))


class SolveParams(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("sampling", C.c_int32), ("update", C.c_int32), ("lanes", C.c_int32),
        ("in_flight", C.c_int64), ("tol", C.c_double), ("x_ref", C.c_void_p),
        ("check_every", C.c_int32), ("refine", C.c_int32), ("inner_sweeps", C.c_int64),
        ("stream_id", C.c_uint32), ("trace", C.c_int32), ("ticket0", C.c_int64),
        ("cancel", C.c_void_p), ("history", C.c_void_p), ("history_cap", C.c_int64),
        ("iter_dtype", C.c_int32), ("order", C.c_int32), ("pipeline", C.c_int32), ("skip_resid", C.c_int32),
    ]


class SolveStats(C.Structure):
    _fields_ = [
        ("sweeps_done", C.c_int64), ("row_updates", C.c_int64), ("next_ticket", C.c_int64),
        ("history_len", C.c_int64), ("in_flight", C.c_int64), ("lanes", C.c_int32),
        ("outer_iters", C.c_int32), ("pipelined", C.c_int32), ("reserved", C.c_int32),
        ("seconds", C.c_double), ("sweep_seconds", C.c_double),
        ("rows_per_s", C.c_double), ("final_err", C.c_double), ("tau_design", C.c_double),
        ("tau_obs_mean", C.c_double), ("tau_obs_max", C.c_double), ("window_ns_mean", C.c_double),
        ("window_ns_max", C.c_double), ("tau_samples", C.c_int64), ("lambda_max_est", C.c_double),
        ("tau_max_corollary", C.c_double), ("final_resid", C.c_double), ("lambda_source", C.c_int32),
        ("reserved2", C.c_int32),
    ]


class SystemInfo(C.Structure):
    _fields_ = [
        ("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64), ("mu", C.c_int64), ("nu", C.c_int64),
        ("fixed_nnz", C.c_int64), ("record_stride", C.c_int64), ("device_bytes", C.c_int64),
        ("vals_dtype", C.c_int32), ("iter_dtype", C.c_int32), ("fro2", C.c_double),
        ("lambda_mp", C.c_double), ("record_bytes_per_row", C.c_int64),
        ("max_col_norm2", C.c_double), ("default_in_flight", C.c_int64),
        ("iterate_stride", C.c_int64), ("tuned_in_flight", C.c_int64),
    ]


class ServerConfig(C.Structure):
    _fields_ = [
        ("budget_bytes", C.c_int64), ("max_slots", C.c_int32), ("inner_sweeps", C.c_int32),
        ("max_workers", C.c_int64), ("max_rounds", C.c_int32), ("use_graph", C.c_int32),
        ("gamma", C.c_double), ("pinned_bytes", C.c_int64), ("lanes", C.c_int32), ("pipe_workers", C.c_int32),
        ("pipe_lanes", C.c_int32), ("fixed_rounds", C.c_int32), ("order", C.c_int32),
        ("pinned_wait_ms", C.c_int32),
    ]


class RequestStats(C.Structure):
    _fields_ = [
        ("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64), ("in_flight", C.c_int64),
        ("sweeps", C.c_int64), ("rounds", C.c_int32), ("status", C.c_int32),
        ("rel_residual", C.c_double), ("t_submit", C.c_double), ("t_admit", C.c_double),
        ("t_done", C.c_double),
    ]


class ServerStats(C.Structure):
    _fields_ = [
        ("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
        ("active", C.c_int64), ("queued", C.c_int64), ("rounds", C.c_int64),
        ("row_updates", C.c_int64), ("arena_used", C.c_int64), ("gpu_seconds", C.c_double),
        ("round_workers", C.c_int64), ("round_systems", C.c_int64), ("pipelined_rounds", C.c_int64),
        ("lanes", C.c_int32), ("pipe_lanes", C.c_int32), ("lanes_tuning", C.c_int32),
        ("buckets_untuned", C.c_int32), ("pageable_uploads", C.c_int64),
    ]


_lib = None


def library_path() -> Path:
    return LIB_PATH


def lib():
    """Load libasyrk.so (raises LibraryMissing when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise LibraryMissing(f"{LIB_PATH} is not built; run `python -m paper_1401_4780_amd.build`")
    # torch ships its own HIP runtime under the same soname: loaded first, it
    # serves this library too.  Loaded after the system runtime, it would be a
    # second runtime in the process, and torch would then see no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(str(LIB_PATH))
    P, i64, u64, u32, i32, dbl = C.c_void_p, C.c_int64, C.c_uint64, C.c_uint32, C.c_int32, C.c_double
    L.asyrk_abi_version.restype = C.c_int
    L.asyrk_status_string.restype = C.c_char_p
    L.asyrk_status_string.argtypes = [C.c_int]
    L.asyrk_last_error_message.restype = C.c_char_p
    L.asyrk_solve_params_init.argtypes = [P]
    L.asyrk_solve_params_init.restype = None
    L.asyrk_create.argtypes = [P, i64, i64, P, P, P, i32, P, i32, P]
    L.asyrk_create_augmented.argtypes = [P, i64, i64, P, P, P, i32, P, dbl, dbl, i32, P]
    L.asyrk_augmented_solution.argtypes = [P, P, P]
    L.asyrk_destroy.argtypes = [P]
    L.asyrk_set_rhs.argtypes = [P, P]
    L.asyrk_system_info_get.argtypes = [P, P]
    L.asyrk_records_get.argtypes = [P, P, i64, P]
    L.asyrk_solve.argtypes = [P, P, dbl, i64, u64, P, P]
    L.asyrk_residual.argtypes = [P, P, P, P]
    L.asyrk_sample_rows.argtypes = [P, u64, u32, i32, i64, i64, P, P]
    L.asyrk_lambda_max.argtypes = [P, i32, u64, P, P]
    L.asyrk_lambda_max_noalloc.argtypes = [P, i32, u64, P, P]
    L.asyrk_autotune.argtypes = [P, dbl, i32, i64, P, P, P]
    L.asyrk_probe_copy.argtypes = [i64, i32, P]
    L.asyrk_probe_scatter.argtypes = [i64, i64, i32, i32, i32, P]
    L.asyrk_server_config_init.argtypes = [P]
    L.asyrk_server_config_init.restype = None
    L.asyrk_server_create.argtypes = [P, P]
    L.asyrk_server_destroy.argtypes = [P]
    L.asyrk_server_submit.argtypes = [P, i64, i64, P, P, P, P, dbl, u64, P]
    L.asyrk_server_progress.argtypes = [P, P, P]
    L.asyrk_server_run.argtypes = [P, P]
    L.asyrk_server_poll.argtypes = [P, i64, P, P]
    L.asyrk_server_stats_get.argtypes = [P, P]
    L.asyrk_server_take_completed.argtypes = [P, P, i64, P]
    L.asyrk_now.argtypes = []
    L.asyrk_now.restype = dbl
    for name in ("asyrk_create", "asyrk_create_augmented", "asyrk_augmented_solution", "asyrk_destroy", "asyrk_set_rhs", "asyrk_system_info_get",
                 "asyrk_records_get",
                 "asyrk_solve", "asyrk_residual", "asyrk_sample_rows", "asyrk_lambda_max", "asyrk_lambda_max_noalloc",
                 "asyrk_probe_copy", "asyrk_probe_scatter", "asyrk_autotune", "asyrk_server_create",
                 "asyrk_server_destroy", "asyrk_server_submit", "asyrk_server_progress",
                 "asyrk_server_poll", "asyrk_server_stats_get", "asyrk_server_take_completed",
                 "asyrk_server_run"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc != 0:
        detail = lib().asyrk_last_error_message().decode() if rc in (3, 4) else ""
        raise AsyrkError(rc, where, detail)


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _ptr(a):
    """Raw pointer of a contiguous numpy array or torch tensor (None passes through)."""
    if a is None:
        return None
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr()
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return a.ctypes.data


def _vals_dtype(val, dtype):
    if dtype is not None:
        return {"f64": F64, "f32": F32, "bf16": BF16}[dtype]
    name = str(val.dtype)
    if name.endswith("float64"):
        return F64
    if name.endswith("float32"):
        return F32
    if name.endswith("bfloat16") or name.endswith("uint16") or name.endswith("int16"):
        return BF16
    raise TypeError(f"unsupported value dtype {val.dtype}")


def _expect(a, device, kind, name):
    """Check that an array matches the system's memory kind and element type."""
    if device:
        if not _is_torch(a) or not a.is_cuda:
            raise TypeError(f"{name}: expected a CUDA tensor")
    elif _is_torch(a) or not isinstance(a, np.ndarray):
        raise TypeError(f"{name}: expected a numpy array")
    dt = str(a.dtype)
    if not dt.endswith(kind):
        raise TypeError(f"{name}: expected {kind}, got {dt}")


def _numel(a) -> int:
    return int(a.numel()) if _is_torch(a) else int(a.size)


def _expect_len(a, count, name, at_least=False):
    """The C ABI reads `count` elements through the pointer: check they exist."""
    k = _numel(a)
    if k < count or (not at_least and k != count):
        raise ValueError(f"{name}: {k} elements, expected {'at least ' if at_least else ''}{count}")


def _last(a) -> int:
    """Last element of a 1-D integer array or tensor (nnz from row_ptr)."""
    return int(a[-1].item()) if _is_torch(a) else int(a[-1])


class System:
    """A consistent sparse system A x = b resident on the GPU.

    ``row_ptr`` int64[m+1], ``col`` int32[nnz], ``val`` float64/float32 or
    bfloat16 bits (uint16/int16/torch.bfloat16, or pass dtype="bf16"),
    ``b`` float64[m].  All numpy (host) or all torch CUDA tensors (device).
    """

    def __init__(self, row_ptr, col, val, b, *, n=None, dtype=None, stream=None, augmented=None):
        """augmented=(zeta, phi): build the paper's consistent augmented system
        for least squares of an inconsistent A x = b (size n + m); solve it for
        z and read the least-squares x with least_squares_x(z)."""
        L = lib()
        self.device = _is_torch(row_ptr) and row_ptr.is_cuda
        _expect(row_ptr, self.device, "int64", "row_ptr")
        _expect(col, self.device, "int32", "col")
        _expect(b, self.device, "float64", "b")
        self.m = int(row_ptr.shape[0]) - 1
        if self.m >= 1:
            nnz = _last(row_ptr)
            _expect_len(col, max(nnz, 0), "col", at_least=True)
            _expect_len(val, max(nnz, 0), "val", at_least=True)
            _expect_len(b, self.m, "b")
        if n is None:
            n = int(col.max()) + 1 if int(col.shape[0]) else 1
        self.n = int(n)
        self.vals_dtype = _vals_dtype(val, dtype)
        if stream is None and self.device:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        h = C.c_void_p()
        mem = MEM_DEVICE if self.device else MEM_HOST
        if augmented is None:
            rc = L.asyrk_create(C.byref(h), self.m, self.n, _ptr(row_ptr), _ptr(col), _ptr(val),
                                self.vals_dtype, _ptr(b), mem, stream)
            _check(rc, "asyrk_create")
        else:
            zeta, phi = augmented
            rc = L.asyrk_create_augmented(C.byref(h), self.m, self.n, _ptr(row_ptr), _ptr(col), _ptr(val),
                                          self.vals_dtype, _ptr(b), float(zeta), float(phi), mem, stream)
            _check(rc, "asyrk_create_augmented")
            self.a_shape = (self.m, self.n)
            self.m = self.n = self.m + self.n
        self._h = h

    def least_squares_x(self, z, out=None):
        """The least-squares solution of the original A x = b from the augmented
        unknown z (asyrk_augmented_solution); a system built with augmented=..."""
        if not hasattr(self, "a_shape"):
            raise TypeError("least_squares_x: not an augmented system")
        _expect(z, self.device, "float64", "z")
        _expect_len(z, self.n, "z")
        n = self.a_shape[1]
        if out is None:
            if self.device:
                import torch
                out = torch.empty(n, dtype=torch.float64, device=z.device)
            else:
                out = np.empty(n, dtype=np.float64)
        _expect(out, self.device, "float64", "out")
        _expect_len(out, n, "out")
        _check(lib().asyrk_augmented_solution(self._h, _ptr(z), _ptr(out)), "asyrk_augmented_solution")
        return out

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            lib().asyrk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- queries
    def info(self) -> dict:
        inf = SystemInfo()
        _check(lib().asyrk_system_info_get(self._h, C.byref(inf)), "asyrk_system_info_get")
        return {f: getattr(inf, f) for f, _ in SystemInfo._fields_}

    def records(self) -> np.ndarray:
        """The packed row records as the sweep reads them (uint8), copied to
        the host, for checking the setup."""
        size = C.c_int64(0)
        _check(lib().asyrk_records_get(self._h, None, 0, C.byref(size)), "asyrk_records_get")
        out = np.empty(size.value, np.uint8)
        _check(lib().asyrk_records_get(self._h, out.ctypes.data, size.value, None), "asyrk_records_get")
        return out

    def set_rhs(self, b):
        _expect(b, self.device, "float64", "b")
        _expect_len(b, self.m, "b")
        _check(lib().asyrk_set_rhs(self._h, _ptr(b)), "asyrk_set_rhs")

    def residual(self, x, r_out=None) -> float:
        """||b - A x||^2 in FP64 (r_out, if given, receives b - A x)."""
        _expect(x, self.device, "float64", "x")
        _expect_len(x, self.n, "x")
        if r_out is not None:
            _expect(r_out, self.device, "float64", "r_out")
            _expect_len(r_out, self.m, "r_out")
        v = C.c_double()
        _check(lib().asyrk_residual(self._h, _ptr(x), _ptr(r_out), C.byref(v)), "asyrk_residual")
        return v.value

    def sample_rows(self, seed, count, ticket0=0, stream_id=0, uniform=False, rows_out=None,
                    coords_out=None):
        """Rows (and Algorithm 1 positions) the device sampler draws for tickets."""
        if rows_out is None:
            if self.device:
                import torch
                rows_out = torch.empty(count, dtype=torch.int32, device="cuda")
            else:
                rows_out = np.empty(count, dtype=np.int32)
        _expect(rows_out, self.device, "int32", "rows_out")
        _expect_len(rows_out, count, "rows_out", at_least=True)
        if coords_out is not None:
            _expect(coords_out, self.device, "int32", "coords_out")
            _expect_len(coords_out, count, "coords_out", at_least=True)
        _check(lib().asyrk_sample_rows(self._h, seed, stream_id, SAMPLE_UNIFORM if uniform else SAMPLE_NORM2,
                                       ticket0, count, _ptr(rows_out), _ptr(coords_out)),
               "asyrk_sample_rows")
        return rows_out

    def lambda_max(self, iters=60, seed=0, noalloc=False):
        """(lambda_max(A^T A) by power iteration, Corollary 1's largest tau or -1).
        noalloc=True: the allocation-free entry point (fixed scratch)."""
        lam, tau = C.c_double(), C.c_double()
        fn = lib().asyrk_lambda_max_noalloc if noalloc else lib().asyrk_lambda_max
        _check(fn(self._h, iters, seed, C.byref(lam), C.byref(tau)),
               "asyrk_lambda_max_noalloc" if noalloc else "asyrk_lambda_max")
        return lam.value, tau.value

    def autotune(self, gamma=1.0, iter_dtype=None, in_flight=0):
        """Time one sweep per lane-group width and worker loop; the fastest pair
        becomes the default at this R (in_flight = 0: the default R; "auto":
        the autotuner picks R too, see info()["tuned_in_flight"]).  Returns
        (best G, loop, {(G, loop): rows/s}) at that R, loop 0 plain,
        1 pipelined, 2 batched."""
        if in_flight == "auto":
            in_flight = -1
        best, pipe = C.c_int32(), C.c_int32()
        rates = (C.c_double * 21)()
        _check(lib().asyrk_autotune(self._h, float(gamma), {None: -1, "f32": F32, "f64": F64}[iter_dtype],
                                    int(in_flight), C.byref(best), C.byref(pipe), rates), "asyrk_autotune")
        keys = [(g, p) for p in (0, 1, 2) for g in (1, 2, 4, 8, 16, 32, 64)]
        return best.value, pipe.value, dict(zip(keys, list(rates)))

    # -- the method
    def solve(self, x, gamma=1.0, sweeps=1, seed=0, *, mode="async", sampling="norm2",
              update="all", lanes=0, in_flight=0, tol=0.0, x_ref=None, check_every=1,
              refine=False, inner_sweeps=0, stream_id=0, trace=False, ticket0=0, cancel=None,
              history=0, iter_dtype=None, order="replacement", pipeline=None, final_resid=True) -> dict:
        """Run from x (float64, overwritten with the result).  Returns the stats
        as a dict with ``status`` ("OK", "NOT_CONVERGED", "DIVERGED" or
        "CANCELLED") and, when ``history`` > 0, the monitored-error history.
        ``pipeline``: None for the library's choice, 0 (or False) the plain
        worker loop, 1 (or True) the pipelined one, 2 the batched one; the
        stats' ``pipelined`` names the loop that ran."""
        _expect(x, self.device, "float64", "x")
        _expect_len(x, self.n, "x")
        if x_ref is not None:
            _expect(x_ref, self.device, "float64", "x_ref")
            _expect_len(x_ref, self.n, "x_ref")
        p = SolveParams()
        lib().asyrk_solve_params_init(C.byref(p))
        p.mode = {"async": ASYNC, "replay": REPLAY}[mode]
        p.sampling = {"norm2": SAMPLE_NORM2, "uniform": SAMPLE_UNIFORM}[sampling]
        p.update = {"all": UPDATE_ALL, "one": UPDATE_ONE}[update]
        p.lanes = lanes
        p.in_flight = in_flight
        p.tol = tol
        p.x_ref = _ptr(x_ref)
        p.check_every = check_every
        p.refine = int(bool(refine))
        p.inner_sweeps = inner_sweeps
        p.stream_id = stream_id
        p.trace = int(bool(trace))
        p.ticket0 = ticket0
        p.iter_dtype = {None: -1, "f32": F32, "f64": F64}[iter_dtype]
        p.order = {"replacement": 0, "slices": 1}[order]
        p.pipeline = -1 if pipeline is None else int(pipeline)  # False/True/0/1/2; others are rejected
        p.skip_resid = 0 if final_resid else 1
        if cancel is not None:
            if not (isinstance(cancel, np.ndarray) and cancel.dtype == np.int32):
                raise TypeError("cancel: expected a numpy int32 array")
            p.cancel = cancel.ctypes.data
        hist = None
        if history:
            hist = np.zeros(int(history), dtype=np.float64)
            p.history = hist.ctypes.data
            p.history_cap = hist.size
        st = SolveStats()
        rc = lib().asyrk_solve(self._h, _ptr(x), float(gamma), int(sweeps), int(seed), C.byref(p),
                               C.byref(st))
        if rc != 0 and rc not in _SOFT:
            _check(rc, "asyrk_solve")
        out = {f: getattr(st, f) for f, _ in SolveStats._fields_}
        out["status"] = STATUS[rc]
        if hist is not None:
            out["history"] = hist[: st.history_len].copy()
        for k in ("final_err", "final_resid"):
            if not math.isfinite(out[k]):
                out[k] = float("nan")
        return out


def now() -> float:
    """The server's clock (steady clock, seconds)."""
    return lib().asyrk_now()


class Server:
    """Continuous-batching solve server (asyrk_server_*): submit systems with
    FP32 values from any thread, drive rounds with progress() from one thread
    or with start() (the library's own round loop on a background thread),
    collect results with poll()."""

    def __init__(self, **cfg):
        L = lib()
        c = ServerConfig()
        L.asyrk_server_config_init(C.byref(c))
        for k, v in cfg.items():
            if k == "use_graph":
                v = int(bool(v))
            setattr(c, k, v)
        h = C.c_void_p()
        _check(L.asyrk_server_create(C.byref(h), C.byref(c)), "asyrk_server_create")
        self._h = h
        self.config = {f: getattr(c, f) for f, _ in ServerConfig._fields_}
        self._runner = None
        self._n_of = {}  # request id -> n (the length poll writes)

    def start(self):
        """Run rounds on a background thread (asyrk_server_run: the loop is
        native, so it runs outside the GIL) until stop()."""
        import threading
        if self._runner is not None:
            raise RuntimeError("the round loop is already running")
        self._stop = C.c_int32(0)
        self._run_rc = None

        def body():
            self._run_rc = lib().asyrk_server_run(self._h, C.byref(self._stop))

        self._runner = threading.Thread(target=body, daemon=True)
        self._runner.start()

    def stop(self):
        """End the round loop started by start(); raises if it ended on an error."""
        if getattr(self, "_runner", None) is None:
            return
        self._stop.value = 1
        self._runner.join()
        self._runner = None
        _check(self._run_rc, "asyrk_server_run")

    def close(self):
        if getattr(self, "_h", None):
            try:
                self.stop()
            finally:
                lib().asyrk_server_destroy(self._h)
                self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, row_ptr, col, val, b, *, n, tol=1e-8, seed=0) -> int:
        for a, kind, name in ((row_ptr, "int64", "row_ptr"), (col, "int32", "col"),
                              (val, "float32", "val"), (b, "float64", "b")):
            _expect(a, False, kind, name)
        m = int(row_ptr.shape[0]) - 1
        if m >= 1:
            nnz = max(int(row_ptr[-1]), 0)
            _expect_len(col, nnz, "col", at_least=True)
            _expect_len(val, nnz, "val", at_least=True)
            _expect_len(b, m, "b")
        rid = C.c_int64()
        _check(lib().asyrk_server_submit(self._h, m, int(n), _ptr(row_ptr), _ptr(col),
                                         _ptr(val), _ptr(b), float(tol), int(seed), C.byref(rid)),
               "asyrk_server_submit")
        self._n_of[rid.value] = int(n)
        return rid.value

    def progress(self):
        """One round; returns (active, queued) afterwards.  Not while start()'s
        loop runs (one thread runs rounds at a time)."""
        if getattr(self, "_runner", None) is not None:
            raise RuntimeError("the round loop started by start() is running; call stop() first")
        a, q = C.c_int32(), C.c_int32()
        _check(lib().asyrk_server_progress(self._h, C.byref(a), C.byref(q)), "asyrk_server_progress")
        return a.value, q.value

    def poll(self, request_id, n=None):
        """None while pending; else (status, stats dict, x) and the request is
        released.  x (length n, the request's column count) is returned when n
        is given."""
        rid = int(request_id)
        known = self._n_of.get(rid)
        if n is not None and known is not None and int(n) != known:
            raise ValueError(f"request {rid} has n = {known}, not {n}")
        st = RequestStats()
        x = np.empty(known, dtype=np.float64) if (n is not None and known is not None) else None
        rc = lib().asyrk_server_poll(self._h, rid, _ptr(x), C.byref(st))
        if rc == 9:
            return None
        if rc not in (0, 5, 6):
            _check(rc, "asyrk_server_poll")
        self._n_of.pop(rid, None)
        return STATUS[rc], {f: getattr(st, f) for f, _ in RequestStats._fields_}, x

    def take_completed(self, cap=4096):
        """Ids of requests finished since the last call."""
        ids = np.empty(cap, dtype=np.int64)
        cnt = C.c_int64()
        _check(lib().asyrk_server_take_completed(self._h, _ptr(ids), cap, C.byref(cnt)),
               "asyrk_server_take_completed")
        return ids[: cnt.value].tolist()

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().asyrk_server_stats_get(self._h, C.byref(st)), "asyrk_server_stats_get")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}


def probe_copy(nbytes=1 << 30, iters=20) -> float:
    """Streaming copy bandwidth in GB/s (read + write bytes)."""
    v = C.c_double()
    _check(lib().asyrk_probe_copy(nbytes, iters, C.byref(v)), "asyrk_probe_copy")
    return v.value


def probe_scatter(n, count, dtype="f32", kind="load", iters=10) -> float:
    """Random 4/8-byte accesses per second over a table of n elements
    (kind "load": agent-coherent loads, "atomic": no-return atomic adds)."""
    v = C.c_double()
    _check(lib().asyrk_probe_scatter(n, count, {"f32": F32, "f64": F64}[dtype],
                                     {"load": 0, "atomic": 1}[kind], iters, C.byref(v)),
           "asyrk_probe_scatter")
    return v.value
