"""Setup of systems handed over in device memory (validation, row weights and
column statistics, records written on the device) against the host setup of
the same arrays, through the C ABI.

Bars: the record images are byte-identical (headers, units, padding); the
statistics that are exact sums or counts are equal; the largest column norm,
summed by atomics in any order on the device, agrees to 1e-13 relative (the
rounding of at most a few hundred FP64 additions); invalid inputs give the
host's status.  The host setup itself is pinned to the oracle by the sampler
and replay tests.
"""
import sys

import numpy as np
import pytest

import paper_1401_4780_amd as P
import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _ragged(m, n, seed, dtype, long_rows=0):
    rng = np.random.default_rng(seed)
    lens = rng.integers(1, 38, m)
    if long_rows:
        lens[rng.choice(m, long_rows, replace=False)] = 300
    return synth.ragged_rows(m, n, lens, seed=seed, dtype=dtype)


CASES = {
    # equal rows: 20 FP32 entries -> 176 raw bytes padded to 192
    "f32_fixed_pad64": lambda: synth.uniform_rows(3001, 800, 20, seed=1, dtype="f32"),
    "f32_fixed_raw": lambda: synth.uniform_rows(1500, 500, 7, seed=2, dtype="f32"),
    "f64_fixed": lambda: synth.uniform_rows(2000, 400, 9, seed=3, dtype="f64"),
    "bf16_fixed": lambda: synth.uniform_rows(1700, 300, 12, seed=4, dtype="bf16"),
    "f64_ragged_long": lambda: _ragged(2500, 700, 5, "f64", long_rows=3),
    "f32_ragged": lambda: _ragged(4099, 1000, 6, "f32"),
    "bf16_ragged_long": lambda: _ragged(1300, 600, 7, "bf16", long_rows=2),
    "one_row": lambda: synth.ragged_rows(1, 5, [3], seed=8, dtype="f64"),
}

EXACT = ("m", "n", "nnz", "mu", "nu", "fixed_nnz", "record_stride", "vals_dtype", "fro2",
         "record_bytes_per_row", "iterate_stride")


@pytest.mark.parametrize("case", sorted(CASES))
def test_device_setup_matches_host_setup(case):
    s = CASES[case]()
    _say(f"device setup {case} m={s.m} n={s.n} nnz={s.nnz}")
    host = P.System(s.row_ptr, s.col, s.val, s.b, n=s.n, dtype=s.dtype)
    dev = P.System(_dev(s.row_ptr), _dev(s.col), _dev(s.val), _dev(s.b), n=s.n, dtype=s.dtype)
    ih, idv = host.info(), dev.info()
    for k in EXACT:
        assert ih[k] == idv[k], k
    assert abs(ih["max_col_norm2"] - idv["max_col_norm2"]) <= 1e-13 * ih["max_col_norm2"]
    rh, rd = host.records(), dev.records()
    assert rh.shape == rd.shape
    diff = np.flatnonzero(rh != rd)
    assert diff.size == 0, f"{diff.size} bytes differ, first at {diff[:8]}"
    # the same records drive the same replay, bit for bit
    xh, xd = np.zeros(s.n), _dev(np.zeros(s.n))
    host.solve(xh, 1.0, 2, 11, mode="replay")
    dev.solve(xd, 1.0, 2, 11, mode="replay")
    assert np.array_equal(xh, xd.cpu().numpy())
    host.close()
    dev.close()


def _status(fn):
    try:
        fn().close()
        return "OK"
    except P.AsyrkError as e:
        return e.name


def _bad_inputs():
    s = synth.uniform_rows(600, 200, 6, seed=9, dtype="f32")
    out = {}
    c = s.col.copy(); c[6 * 17 + 2] = 200                       # column out of range
    out["col_range"] = (s.row_ptr, c, s.val, s.b)
    c = s.col.copy(); c[6 * 40 + 3] = c[6 * 40 + 2]              # repeated column
    out["col_repeat"] = (s.row_ptr, c, s.val, s.b)
    c = s.col.copy(); c[6 * 41 + 1], c[6 * 41 + 2] = c[6 * 41 + 2], c[6 * 41 + 1]   # unsorted
    out["col_order"] = (s.row_ptr, c, s.val, s.b)
    c = s.col.copy(); c[6 * 3] = -1                              # negative column
    out["col_negative"] = (s.row_ptr, c, s.val, s.b)
    v = s.val.copy(); v[6 * 500 + 4] = np.nan
    out["val_nan"] = (s.row_ptr, s.col, v, s.b)
    v = s.val.copy(); v[6 * 599 + 5] = np.inf
    out["val_inf"] = (s.row_ptr, s.col, v, s.b)
    b = s.b.copy(); b[123] = np.nan
    out["b_nan"] = (s.row_ptr, s.col, s.val, b)
    v = s.val.copy(); v[6 * 300:6 * 301] = 0.0                   # a row of zeros
    out["zero_row"] = (s.row_ptr, s.col, v, s.b)
    rp = s.row_ptr.copy(); rp[250:] -= 6                         # an empty row (nnz drops by 6)
    out["empty_row"] = (rp, s.col, s.val, s.b)
    rp = s.row_ptr.copy(); rp[10], rp[11] = rp[11], rp[10]       # decreasing row_ptr
    out["row_ptr_order"] = (rp, s.col, s.val, s.b)
    rp = s.row_ptr.copy(); rp[0] = 1
    out["row_ptr_start"] = (rp, s.col, s.val, s.b)
    return out


@pytest.mark.parametrize("case", sorted(_bad_inputs()))
def test_device_setup_statuses_match_host(case):
    rp, c, v, b = _bad_inputs()[case]
    _say(f"device setup status {case}")
    h = _status(lambda: P.System(rp, c, v, b, n=200, dtype="f32"))
    d = _status(lambda: P.System(_dev(rp), _dev(c), _dev(v), _dev(b), n=200, dtype="f32"))
    assert h == d and h in ("INVALID_ARG", "ZERO_ROW"), (h, d)
    if case in ("zero_row", "empty_row"):
        assert d == "ZERO_ROW"
