"""CPU oracle for the asynchronous randomized Kaczmarz sweep.

TEST INFRASTRUCTURE ONLY: the plain, slow, sequential FP64 reference that the
GPU library is checked against.  Only ``tests/``, the smoke check and the
CPU-baseline leg of ``bench.py`` may import it; the GPU library never does,
and the two share no code.

The arithmetic lives in ``rk_oracle.c`` (plain C, ``-O2 -ffp-contract=off``,
single thread); this module only builds it with gcc and marshals numpy arrays.
Every matrix argument is CSR with float64 values (the stored values promoted
exactly to float64).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "rk_oracle.c"
_BUILD = _HERE / "_build"
_LIB_PATH = _BUILD / "librk_oracle.so"
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared"]

_lib = None

ORC_OK, ORC_ERR_ARG, ORC_ERR_ZERO_ROW, ORC_ERR_NOMEM = 0, 1, 2, 3


class OracleError(RuntimeError):
    pass


def build() -> Path:
    """Compile rk_oracle.c into oracle/_build/librk_oracle.so (always rebuilds)."""
    _BUILD.mkdir(exist_ok=True)
    tmp = _LIB_PATH.with_suffix(".so.tmp%d" % os.getpid())
    cmd = ["gcc", *CFLAGS, str(_SRC), "-o", str(tmp), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists() or _LIB_PATH.stat().st_mtime < _SRC.stat().st_mtime:
        build()
    lib = C.CDLL(str(_LIB_PATH))
    P = C.c_void_p
    i64, u64, u32, i32, f64 = C.c_int64, C.c_uint64, C.c_uint32, C.c_int, C.c_double
    lib.orc_philox4x32_10.argtypes = [P, P, P]
    lib.orc_philox4x32_10.restype = None
    lib.orc_row_weights.argtypes = [i64, P, P, P]
    lib.orc_row_weights.restype = i64
    lib.orc_alias_build.argtypes = [i64, P, P, P]
    lib.orc_alias_build.restype = i32
    lib.orc_sample_rows.argtypes = [i64, u64, u32, P, P, i64, i64, P, P]
    lib.orc_sample_rows.restype = i32
    lib.orc_residual.argtypes = [i64, P, P, P, P, P, P]
    lib.orc_residual.restype = f64
    lib.orc_rk_run.argtypes = [i64, i64, P, P, P, P, P, f64, u64, u32, i32, i32, i64, i64, i64,
                               i64, P, P, P, P, i32, i64]
    lib.orc_slice_order.argtypes = [i64, i64, u64, i64, P]
    lib.orc_slice_order.restype = i32
    lib.orc_rk_run.restype = i32
    lib.orc_rk_apply_rows.argtypes = [i64, i64, P, P, P, P, P, f64, P, P, i64]
    lib.orc_rk_apply_rows.restype = i32
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _check(rc):
    if rc != ORC_OK:
        raise OracleError({1: "invalid argument", 2: "zero row", 3: "out of memory"}.get(rc, rc))


# --------------------------------------------------------------------------

def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block: 4 x uint32 counter, 2 x uint32 key -> 4 x uint32."""
    lib = _load()
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def row_weights(row_ptr, val) -> np.ndarray:
    """w_i = ||a_i||^2 summed in CSR order; raises on a zero row."""
    lib = _load()
    rp = _c(row_ptr, np.int64)
    v = _c(val, np.float64)
    m = rp.size - 1
    w = np.zeros(m)
    bad = lib.orc_row_weights(m, _p(rp), _p(v), _p(w))
    if bad >= 0:
        raise OracleError(f"zero row {bad}")
    return w


def alias_build(w):
    """Vose alias table over weights w: (thresholds uint64 in [0, 2^32], alias int32)."""
    lib = _load()
    w = _c(w, np.float64)
    m = w.size
    t = np.zeros(m, dtype=np.uint64)
    a = np.zeros(m, dtype=np.int32)
    _check(lib.orc_alias_build(m, _p(w), _p(t), _p(a)))
    return t, a


def sample_rows(m, seed, count, ticket0=0, stream=0, thresh=None, alias=None, with_u3=False):
    """Rows drawn for tickets ticket0 .. ticket0+count-1 (uniform when thresh is None)."""
    lib = _load()
    rows = np.zeros(count, dtype=np.int32)
    u3 = np.zeros(count, dtype=np.uint32) if with_u3 else None
    t = None if thresh is None else _c(thresh, np.uint64)
    a = None if alias is None else _c(alias, np.int32)
    _check(lib.orc_sample_rows(m, seed, stream, _p(t), _p(a), ticket0, count, _p(rows), _p(u3)))
    return (rows, u3) if with_u3 else rows


def residual(row_ptr, col, val, b, x, want_r=False):
    """||b - A x||^2 (and r = b - A x when want_r)."""
    lib = _load()
    rp = _c(row_ptr, np.int64)
    cl = _c(col, np.int32)
    v = _c(val, np.float64)
    bb = _c(b, np.float64)
    xx = _c(x, np.float64)
    m = rp.size - 1
    r = np.zeros(m) if want_r else None
    n2 = lib.orc_residual(m, _p(rp), _p(cl), _p(v), _p(bb), _p(xx), _p(r))
    return (n2, r) if want_r else n2


def slice_order(m, workers, seed, sweep) -> np.ndarray:
    """Row order of sweep ``sweep`` in the slice scheme with ``workers`` slices."""
    lib = _load()
    out = np.zeros(m, dtype=np.int32)
    _check(lib.orc_slice_order(m, workers, seed, sweep, _p(out)))
    return out


def rk_run(row_ptr, col, val, b, n, x0, gamma, nsteps, seed, *, stream=0, uniform=False,
           update_one=False, tau=0, ticket0=0, curve_every=0, x_ref=None, want_rows=False,
           slices=False, workers=1, want_res=True):
    """Sequential RK (eq. (2) with step length gamma) for ``nsteps`` tickets.

    Returns a dict with ``x`` and, as requested, ``err`` (||x-x_ref||/||x_ref||),
    ``res`` (||Ax-b||/||b||, unless ``want_res`` is false) sampled every
    ``curve_every`` steps (index 0 is the start point) and ``rows`` (the row
    drawn for every ticket).
    """
    lib = _load()
    rp = _c(row_ptr, np.int64)
    cl = _c(col, np.int32)
    v = _c(val, np.float64)
    bb = _c(b, np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    m = rp.size - 1
    npts = (nsteps // curve_every + 1) if curve_every > 0 else 0
    err = np.zeros(npts) if (curve_every > 0 and x_ref is not None) else None
    res = np.zeros(npts) if (curve_every > 0 and want_res) else None
    rows = np.zeros(nsteps, dtype=np.int32) if want_rows else None
    xr = None if x_ref is None else _c(x_ref, np.float64)
    rc = lib.orc_rk_run(m, n, _p(rp), _p(cl), _p(v), _p(bb), _p(x), float(gamma), seed, stream,
                        int(uniform), int(update_one), int(tau), int(ticket0), int(nsteps),
                        int(curve_every), _p(xr), _p(err), _p(res), _p(rows), int(slices),
                        int(workers))
    _check(rc)
    out = {"x": x}
    if err is not None:
        out["err"] = err
    if res is not None:
        out["res"] = res
    if rows is not None:
        out["rows"] = rows
    return out


def apply_rows(row_ptr, col, val, b, x0, gamma, rows, coords=None):
    """Apply the eq. (2) projection for the given row sequence (no sampling).

    ``coords`` (optional, same length as rows): position inside the row for
    Algorithm 1's single-coordinate step; -1 means every coordinate.
    """
    lib = _load()
    rp = _c(row_ptr, np.int64)
    cl = _c(col, np.int32)
    v = _c(val, np.float64)
    bb = _c(b, np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    rr = _c(rows, np.int32)
    cc = None if coords is None else _c(coords, np.int32)
    _check(lib.orc_rk_apply_rows(rp.size - 1, x.size, _p(rp), _p(cl), _p(v), _p(bb), _p(x),
                                 float(gamma), _p(rr), _p(cc), rr.size))
    return x


def augmented_system(row_ptr, col, val, b, n, zeta, phi=1.0):
    """The consistent augmented system of the paper's Section "Extension to
    Inconsistent Systems" for least squares min ||A x - b||:

        [ 0      phi A^T ] [x]   [phi A^T b]
        [ A     -zeta I  ] [y] = [    0    ]

    in CSR (float64), unknowns z = (x, y) of length n + m.  From the second
    block y = A x / zeta, and the first gives A^T A x = zeta A^T b, so the
    least-squares solution is x / zeta.  Built with scipy's sparse blocks.
    Returns (row_ptr, col, val, b_aug)."""
    import scipy.sparse as sp
    rp = _c(row_ptr, np.int64)
    m = rp.size - 1
    A = sp.csr_matrix((_c(val, np.float64), _c(col, np.int32), rp), shape=(m, n))
    top = sp.hstack([sp.csr_matrix((n, n)), phi * A.T.tocsr()])
    bot = sp.hstack([A, -zeta * sp.identity(m, format="csr")])
    M = sp.vstack([top, bot]).tocsr()
    M.sort_indices()
    M.eliminate_zeros()
    b_aug = np.concatenate([phi * (A.T @ _c(b, np.float64)), np.zeros(m)])
    return M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.astype(np.float64), b_aug
