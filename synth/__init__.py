"""Seeded synthetic consistent sparse systems ``Ax = b``.

This module builds inputs only.  It holds none of the Kaczmarz arithmetic: it
is shared by the CPU oracle's tests and by the GPU path's tests and benchmark,
and neither of those imports the other.

Recipe (paper, Section "Experiments"): nonzero positions are chosen at random,
their values are N(0,1), and every row is normalized afterwards.  The fixed
count of *distinct* columns per row, the skewed (lognormal length, Zipf
column) variant and the serving stream are the workload shapes this project
measures on; each choice the paper leaves open is documented on the function
that makes it.

Every array that describes the stored matrix is returned in CSR form:

* ``row_ptr``  int64, length m+1, ``row_ptr[0] == 0``
* ``col``      int32, sorted strictly increasing inside each row
* ``val``      the *stored* values: float64, float32, or bfloat16 bit patterns
               (uint16, round-to-nearest-even of the float32 value)
* ``val64``    the stored values promoted exactly to float64
* ``x_star``   float64 solution, ``b = A @ x_star`` in float64 from ``val64``
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "SparseSystem",
    "uniform_rows",
    "skewed_rows",
    "serving_specs",
    "serving_system",
    "poisson_arrivals",
    "ragged_rows",
    "as_dtype",
    "bf16_bits_from_f32",
    "f64_from_bf16_bits",
    "DTYPES",
]

DTYPES = ("f64", "f32", "bf16")


@dataclasses.dataclass
class SparseSystem:
    m: int
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    dtype: str
    val64: np.ndarray
    x_star: np.ndarray
    b: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_nnz(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def dense(self) -> np.ndarray:
        """Dense float64 copy (tiny systems only)."""
        a = np.zeros((self.m, self.n))
        rows = np.repeat(np.arange(self.m), self.row_nnz())
        a[rows, self.col] = self.val64
        return a

    def csr_bytes(self) -> int:
        return self.row_ptr.nbytes + self.col.nbytes + self.val.nbytes


def bf16_bits_from_f32(v: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); return the bits."""
    u = np.ascontiguousarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
    bias = ((u >> np.uint64(16)) & np.uint64(1)) + np.uint64(0x7FFF)
    return ((u + bias) >> np.uint64(16)).astype(np.uint16)


def f64_from_bf16_bits(bits: np.ndarray) -> np.ndarray:
    u = bits.astype(np.uint32) << np.uint32(16)
    return u.view(np.float32).astype(np.float64)


def _store(v64: np.ndarray, dtype: str):
    """Round float64 values to the storage dtype; return (stored, promoted-f64)."""
    if dtype == "f64":
        return v64.copy(), v64.copy()
    f32 = v64.astype(np.float32)
    if dtype == "f32":
        return f32, f32.astype(np.float64)
    if dtype == "bf16":
        bits = bf16_bits_from_f32(f32)
        return bits, f64_from_bf16_bits(bits)
    raise ValueError(f"unknown dtype {dtype!r}")


def _distinct_uniform_cols(rng: np.random.Generator, m: int, n: int, k: int) -> np.ndarray:
    """(m, k) int64 array, each row k distinct columns of [0, n), sorted ascending.

    Rows that draw a repeated column are drawn again until none repeats.
    """
    if k > n:
        raise ValueError("more nonzeros per row than columns")
    if n <= 4 * k or m * n <= 4_000_000:
        # small: take the first k of a random permutation per row
        keys = rng.random((m, n))
        cols = np.argpartition(keys, k - 1, axis=1)[:, :k] if k < n else np.argsort(keys, axis=1)
        cols.sort(axis=1)
        return cols.astype(np.int64)
    cols = rng.integers(0, n, size=(m, k), dtype=np.int64)
    cols.sort(axis=1)
    bad = np.nonzero((np.diff(cols, axis=1) == 0).any(axis=1))[0]
    while bad.size:
        redo = rng.integers(0, n, size=(bad.size, k), dtype=np.int64)
        redo.sort(axis=1)
        cols[bad] = redo
        sub = (np.diff(redo, axis=1) == 0).any(axis=1)
        bad = bad[sub]
    return cols


def _normal_rows_normalized(rng, nnz_total: int, row_ptr: np.ndarray) -> np.ndarray:
    v = rng.standard_normal(nnz_total)
    sq = np.add.reduceat(v * v, row_ptr[:-1]) if nnz_total else np.zeros(0)
    nrm = np.sqrt(sq)
    return v / np.repeat(nrm, np.diff(row_ptr))


def _finish(m, n, row_ptr, col, v64, dtype, rng, x_star=None, x_star_mode="normal"):
    val, val64 = _store(v64, dtype)
    if np.any(val64 == 0.0) and dtype != "f64":
        # an entry that rounded to zero would be a stored zero; re-round upward
        raise RuntimeError("a stored nonzero rounded to zero; change the seed")
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(row_ptr))
    if x_star is None:
        if x_star_mode == "normal":
            x_star = rng.standard_normal(n)
        elif x_star_mode == "range":
            # x* = A^T y rescaled to RMS 1: the minimum-norm solution, reachable from x0 = 0
            y = rng.standard_normal(m)
            x_star = np.bincount(col, weights=val64 * y[rows], minlength=n)
            rms = math.sqrt(float(np.mean(x_star * x_star)))
            x_star = x_star / rms
        else:
            raise ValueError(x_star_mode)
    prod = val64 * x_star[col]
    b = np.add.reduceat(prod, row_ptr[:-1]) if prod.size else np.zeros(m)
    b[np.diff(row_ptr) == 0] = 0.0
    return SparseSystem(m, n, row_ptr, col.astype(np.int32), val, dtype, val64, x_star, b)


def uniform_rows(m: int, n: int, nnz_per_row: int, seed: int, dtype: str = "f32",
                 normalize: bool = True, require_full_columns: bool = True,
                 x_star: np.ndarray | None = None) -> SparseSystem:
    """Every row has exactly ``nnz_per_row`` distinct uniform-random columns.

    Values are N(0,1); rows are scaled to unit norm in float64 and then rounded
    to ``dtype`` (so stored rows are unit norm up to that rounding).  With
    ``normalize=False`` the raw N(0,1) values are kept (row norms then vary,
    which exercises the norm-weighted row sampling).  ``x_star`` ~ N(0,1).

    Draw order for a seed: columns, values, x*.
    """
    rng = np.random.default_rng(seed)
    cols = _distinct_uniform_cols(rng, m, n, nnz_per_row).reshape(-1)
    row_ptr = np.arange(m + 1, dtype=np.int64) * nnz_per_row
    if normalize:
        v64 = _normal_rows_normalized(rng, cols.size, row_ptr)
    else:
        v64 = rng.standard_normal(cols.size)
    if require_full_columns:
        counts = np.bincount(cols, minlength=n)
        if counts.min() == 0:
            raise RuntimeError("an empty column: the solution would not be unique")
    return _finish(m, n, row_ptr, cols, v64, dtype, rng, x_star=x_star)


def _zipf_table(n: int, s: float):
    """Alias table (probability, alias) for P(rank k) proportional to k^-s,
    k = 1..n (index k-1), for O(1) vectorized draws."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    p = w * (n / w.sum())
    prob = np.ones(n)
    alias = np.arange(n)
    small = list(np.nonzero(p < 1.0)[0])
    large = list(np.nonzero(p >= 1.0)[0])
    p = p.tolist()
    while small and large:
        a = small.pop()
        g = large.pop()
        prob[a] = p[a]
        alias[a] = g
        p[g] = (p[g] + p[a]) - 1.0
        (small if p[g] < 1.0 else large).append(g)
    return prob, alias


def _distinct_rows_from_sampler(rng, lengths: np.ndarray, draw) -> np.ndarray:
    """Per row, the first ``lengths[i]`` distinct values of an i.i.d. stream ``draw``.

    Rows are handled in groups of similar length with a pool of draws per row;
    a row whose pool holds too few distinct values is drawn again with a larger
    pool.  Returns the concatenated, per-row sorted column lists.
    """
    m = lengths.size
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    out = np.empty(int(row_ptr[-1]), dtype=np.int64)
    todo = np.arange(m)
    factor = 1.25
    while todo.size:
        lens = lengths[todo]
        g_of = np.floor(np.log2(np.maximum(lens, 1))).astype(np.int64)
        retry = []
        for g in np.unique(g_of):
            idx = todo[g_of == g]
            ln = lengths[idx]
            pool = int(factor * (2 ** (g + 1))) + 16
            draws = draw(rng, (idx.size, pool))
            # first occurrence of each value in draw order
            srt = np.argsort(draws, axis=1, kind="stable")
            sv = np.take_along_axis(draws, srt, axis=1)
            first = np.ones_like(sv, dtype=bool)
            first[:, 1:] = sv[:, 1:] != sv[:, :-1]
            keep = np.zeros_like(first)
            np.put_along_axis(keep, srt, first, axis=1)
            rank = np.cumsum(keep, axis=1)
            ok_rows = rank[:, -1] >= ln
            retry.append(idx[~ok_rows])
            sel = keep & (rank <= ln[:, None]) & ok_rows[:, None]
            r_i, _ = np.nonzero(sel)
            vals = draws[sel]
            # sort each row's values: order by (row, value)
            order = np.lexsort((vals, r_i))
            vals = vals[order]
            r_i = r_i[order]
            good = idx[ok_rows]
            starts = row_ptr[good]
            # position of each value inside its row
            cnt = ln[ok_rows]
            offs = np.repeat(starts, cnt) + (np.arange(vals.size) - np.repeat(np.cumsum(cnt) - cnt, cnt))
            out[offs] = vals
        todo = np.concatenate(retry) if retry else np.zeros(0, dtype=np.int64)
        factor *= 4
    return out


def skewed_rows(m: int, n: int, seed: int, dtype: str = "f32", median: float = 16.0,
                sigma: float = 1.0, lo: int = 4, hi: int = 2000, zipf_s: float = 1.1) -> SparseSystem:
    """Skewed rows: lognormal lengths and Zipf-distributed (hot) columns.

    * nnz_i = clip(round(exp(N(ln median, sigma))), lo, min(hi, n))
    * column ranks 1..n drawn with P(k) proportional to k^-zipf_s (alias
      table, two uniforms per draw), mapped to
      columns through a seeded random permutation (hot columns are scattered),
      distinct within a row (first distinct draws kept).
    * N(0,1) values, rows normalized in float64 then rounded to ``dtype``.
    * the system is rank deficient (empty and singleton columns), so
      ``x_star = A^T y`` (y ~ N(0, I_m)) scaled to RMS 1, the minimum-norm
      solution reachable from x0 = 0.

    Draw order: lengths, permutation, columns, values, y.
    """
    rng = np.random.default_rng(seed)
    lens = np.rint(np.exp(rng.normal(math.log(median), sigma, size=m))).astype(np.int64)
    lens = np.clip(lens, lo, min(hi, n))
    perm = rng.permutation(n).astype(np.int64)
    prob, alias = _zipf_table(n, zipf_s)

    def draw(r, shape):
        k = np.minimum((r.random(shape) * n).astype(np.int64), n - 1)
        ranks = np.where(r.random(shape) < prob[k], k, alias[k])
        return perm[ranks]

    cols = _distinct_rows_from_sampler(rng, lens, draw)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    v64 = _normal_rows_normalized(rng, cols.size, row_ptr)
    return _finish(m, n, row_ptr, cols, v64, dtype, rng, x_star_mode="range")


def as_dtype(s: SparseSystem, dtype: str) -> SparseSystem:
    """The same system stored in another dtype: the float64 values of ``s``
    (which must be stored in f64) rounded to ``dtype``, the same x*, and b
    recomputed from the rounded values.  Equal to generating with ``dtype``
    directly for the same seed, without drawing everything again."""
    if s.dtype != "f64":
        raise ValueError("as_dtype starts from an f64 system")
    val, val64 = _store(s.val64, dtype)
    prod = val64 * s.x_star[s.col]
    b = np.add.reduceat(prod, s.row_ptr[:-1]) if prod.size else np.zeros(s.m)
    b[np.diff(s.row_ptr) == 0] = 0.0
    return SparseSystem(s.m, s.n, s.row_ptr, s.col, val, dtype, val64, s.x_star, b)


def ragged_rows(m: int, n: int, lengths, seed: int, dtype: str = "f64",
                normalize: bool = False) -> SparseSystem:
    """Rows of the given lengths (array of m ints, each in [1, n]) with distinct
    uniform columns and N(0,1) values (left unnormalized by default, so row
    norms differ); x* ~ N(0,1).  For edge cases: single-entry rows, rows far
    longer than the rest, lengths that are not multiples of the record unit.

    Draw order: columns (row by row), values, x*.
    """
    rng = np.random.default_rng(seed)
    lens = np.asarray(lengths, dtype=np.int64)
    if lens.size != m or lens.min() < 1 or lens.max() > n:
        raise ValueError("lengths must hold m values in [1, n]")
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.int64)
    for i in range(m):
        col[row_ptr[i]:row_ptr[i + 1]] = np.sort(rng.choice(n, size=int(lens[i]), replace=False))
    if normalize:
        v64 = _normal_rows_normalized(rng, col.size, row_ptr)
    else:
        v64 = rng.standard_normal(col.size)
    return _finish(m, n, row_ptr, col, v64, dtype, rng)


# --------------------------------------------------------------------------
# Serving stream: many independent small systems
# --------------------------------------------------------------------------

def serving_specs(count: int = 10_000, seed: int = 4, m_lo: int = 1_000, m_hi: int = 200_000,
                  nnz_lo: int = 8, nnz_hi: int = 64):
    """Sizes of the serving stream: m log-uniform in [m_lo, m_hi], n = m // 4.

    Returns an int64 array of shape (count, 2) with (m, n) per request.  Each
    system's contents come from ``serving_system(request_id, m, n, seed)``.
    """
    rng = np.random.default_rng(seed)
    m = np.rint(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), size=count))).astype(np.int64)
    n = m // 4
    return np.stack([m, n], axis=1)


_SG_LIB = None
_HERE = __import__("pathlib").Path(__file__).resolve().parent


def build_serving_gen():
    """Compile serving_gen.c into synth/_build/libservinggen.so (always rebuilds)."""
    import os
    import subprocess
    out = _HERE / "_build"
    out.mkdir(exist_ok=True)
    lib = out / "libservinggen.so"
    tmp = out / f"libservinggen.so.tmp{os.getpid()}"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", str(_HERE / "serving_gen.c"),
                    "-o", str(tmp), "-lm"], check=True)
    os.replace(tmp, lib)
    return lib


def _sg():
    global _SG_LIB
    if _SG_LIB is None:
        import ctypes as C
        lib = _HERE / "_build" / "libservinggen.so"
        if not lib.exists() or lib.stat().st_mtime < (_HERE / "serving_gen.c").stat().st_mtime:
            build_serving_gen()
        L = C.CDLL(str(lib))
        P = C.c_void_p
        L.sg_lengths.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, C.c_int, C.c_int, P]
        L.sg_lengths.restype = C.c_int64
        L.sg_fill.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, P, P, P, P, P, P]
        L.sg_fill.restype = None
        _SG_LIB = L
    return _SG_LIB


def serving_system(request_id: int, m: int, n: int, seed: int = 4,
                   nnz_lo: int = 8, nnz_hi: int = 64) -> SparseSystem:
    """One serving request (FP32 values), generated in C (``serving_gen.c``):
    row lengths uniform in {nnz_lo..nnz_hi} (capped at n), distinct uniform
    columns, N(0,1) values, unit rows, x* ~ N(0,1), b = A x* in FP64.

    Seeded by (seed, request_id) so each request is reproducible on its own;
    the C call releases the GIL, so threads generate requests in parallel.
    """
    L = _sg()
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    nnz = int(L.sg_lengths(seed, request_id, m, n, nnz_lo, nnz_hi, row_ptr.ctypes.data))
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float32)
    val64 = np.empty(nnz, dtype=np.float64)
    x_star = np.empty(n, dtype=np.float64)
    b = np.empty(m, dtype=np.float64)
    L.sg_fill(seed, request_id, m, n, row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data,
              val64.ctypes.data, x_star.ctypes.data, b.ctypes.data)
    return SparseSystem(m, n, row_ptr, col, val, "f32", val64, x_star, b)


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
