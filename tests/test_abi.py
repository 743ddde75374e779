"""The C ABI without a GPU: the library loads, exports every declared symbol,
its structs match the Python binding field for field, and every validation
error is reported before any device call."""
import ctypes as C
import re
import subprocess
from pathlib import Path

import numpy as np
import pytest

import paper_1401_4780_amd as P
import synth

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "asyrk.h"


def _declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(asyrk_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = P.lib()
    names = _declared_functions()
    assert "asyrk_create" in names and "asyrk_solve" in names and "asyrk_residual" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert L.asyrk_abi_version() == 3


def _c_layout(struct, fields):
    src = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){",
           f'printf("%zu\\n", sizeof({struct}));']
    src += [f'printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    src += ["return 0;}"]
    d = Path(__import__("tempfile").mkdtemp())
    (d / "l.c").write_text("\n".join(src))
    subprocess.run(["gcc", "-o", str(d / "l"), str(d / "l.c")], check=True)
    out = subprocess.run([str(d / "l")], capture_output=True, text=True, check=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("cname,pycls", [("asyrk_solve_params", P.SolveParams),
                                         ("asyrk_solve_stats", P.SolveStats),
                                         ("asyrk_system_info", P.SystemInfo),
                                         ("asyrk_server_config", P.ServerConfig),
                                         ("asyrk_request_stats", P.RequestStats),
                                         ("asyrk_server_stats", P.ServerStats)])
def test_struct_layouts_match_binding(cname, pycls):
    fields = [f for f, _ in pycls._fields_]
    lay = _c_layout(cname, fields)
    assert lay[0] == C.sizeof(pycls)
    assert lay[1:] == [getattr(pycls, f).offset for f in fields]


def test_status_strings_and_defaults():
    L = P.lib()
    for code in range(11):
        assert L.asyrk_status_string(code)
    p = P.SolveParams()
    L.asyrk_solve_params_init(C.byref(p))
    assert (p.mode, p.sampling, p.update, p.check_every, p.in_flight, p.lanes) == (0, 0, 0, 1, 0, 0)
    assert p.iter_dtype == -1  # -1 = default; 0 is ASYRK_F64
    assert p.skip_resid == 0 and p.pipeline == -1


def _create(rp, col, val, b, n, dtype=P.F32, mem=P.MEM_HOST):
    h = C.c_void_p()
    rc = P.lib().asyrk_create(C.byref(h), rp.size - 1, n, rp.ctypes.data, col.ctypes.data,
                              val.ctypes.data, dtype, b.ctypes.data, mem, None)
    return rc, h


def _good():
    s = synth.uniform_rows(40, 12, 3, seed=2, dtype="f32", require_full_columns=False)
    return s.row_ptr.copy(), s.col.copy(), s.val.copy(), s.b.copy(), s.n


@pytest.mark.parametrize("case", ["m0", "n0", "rp0", "rp_dec", "col_hi", "col_neg", "col_dup",
                                  "col_unsorted", "val_nan", "val_inf", "b_nan", "dtype", "mem"])
def test_invalid_arguments_rejected_before_device(case):
    rp, col, val, b, n = _good()
    dtype, mem = P.F32, P.MEM_HOST
    m_override = None
    if case == "m0":
        m_override = 0
    elif case == "n0":
        n = 0
    elif case == "rp0":
        rp = rp + 1
    elif case == "rp_dec":
        rp[5], rp[6] = rp[6], rp[5]
    elif case == "col_hi":
        col[7] = n
    elif case == "col_neg":
        col[7] = -1
    elif case == "col_dup":
        col[4] = col[3]
    elif case == "col_unsorted":
        col[3], col[4] = col[4], col[3]
    elif case == "val_nan":
        val[9] = np.nan
    elif case == "val_inf":
        val[9] = np.inf
    elif case == "b_nan":
        b[2] = np.nan
    elif case == "dtype":
        dtype = 7
    elif case == "mem":
        mem = 5
    h = C.c_void_p()
    m = rp.size - 1 if m_override is None else m_override
    rc = P.lib().asyrk_create(C.byref(h), m, n, rp.ctypes.data, col.ctypes.data, val.ctypes.data,
                              dtype, b.ctypes.data, mem, None)
    assert P.STATUS[rc] == "INVALID_ARG"
    assert h.value is None


@pytest.mark.parametrize("case", ["empty_row", "zero_values"])
def test_zero_row_rejected(case):
    rp, col, val, b, n = _good()
    if case == "zero_values":
        val[rp[3]:rp[4]] = 0.0
        rc, _ = _create(rp, col, val, b, n)
    else:
        # row 3 loses its entries
        keep = np.ones(col.size, bool)
        keep[rp[3]:rp[4]] = False
        k = rp[4] - rp[3]
        rp2 = rp.copy()
        rp2[4:] -= k
        rc, _ = _create(rp2, col[keep].copy(), val[keep].copy(), b, n)
    assert P.STATUS[rc] == "ZERO_ROW"


def test_null_handles_rejected():
    L = P.lib()
    x = np.zeros(4)
    v = C.c_double()
    assert P.STATUS[L.asyrk_solve(None, x.ctypes.data, 1.0, 1, 0, None, None)] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_residual(None, x.ctypes.data, None, C.byref(v))] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_create(None, 1, 1, None, None, None, 0, None, 0, None)] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_create_augmented(None, 1, 1, None, None, None, 0, None, 1.0, 1.0, 0,
                                             None)] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_lambda_max(None, 5, 0, C.byref(v), None)] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_lambda_max_noalloc(None, 5, 0, C.byref(v), None)] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_augmented_solution(None, x.ctypes.data, x.ctypes.data)] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_destroy(None)] == "OK"
    assert P.STATUS[L.asyrk_probe_copy(0, 1, C.byref(v))] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_server_create(None, None)] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_server_progress(None, None, None)] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_server_poll(None, 1, None, None)] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_server_take_completed(None, None, 0, None)] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_server_run(None, None)] == "INVALID_ARG"
    size = C.c_int64(-1)
    assert P.STATUS[L.asyrk_records_get(None, None, 0, C.byref(size))] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_set_rhs(None, x.ctypes.data)] == "INVALID_ARG"
    assert P.STATUS[L.asyrk_server_destroy(None)] == "OK"


def test_server_config_validation():
    L = P.lib()
    c = P.ServerConfig()
    L.asyrk_server_config_init(C.byref(c))
    assert c.budget_bytes == 64 << 30 and c.use_graph == 1 and c.max_workers == 65536
    assert c.inner_sweeps == 8 and c.pinned_bytes == 4 << 30 and c.lanes == 4 and c.pipe_workers == 8192 and c.pipe_lanes == 16 and c.fixed_rounds == 0 and c.order == 1
    assert c.pinned_wait_ms == 1000
    for field, bad in (("gamma", 2.0), ("max_slots", 0), ("inner_sweeps", 0), ("budget_bytes", 10),
                       ("pinned_bytes", -1), ("lanes", 16), ("lanes", 2), ("pipe_workers", -1), ("pipe_lanes", 2), ("pipe_lanes", 64), ("fixed_rounds", 2), ("order", 2), ("order", -1), ("pinned_wait_ms", -1)):
        d = P.ServerConfig()
        L.asyrk_server_config_init(C.byref(d))
        setattr(d, field, bad)
        h = C.c_void_p()
        assert P.STATUS[L.asyrk_server_create(C.byref(h), C.byref(d))] == "INVALID_ARG"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(P, "LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(P, "_lib", None)
    with pytest.raises(P.LibraryMissing):
        P.lib()


def test_binding_type_checks():
    rp, col, val, b, n = _good()
    with pytest.raises(TypeError):
        P.System(rp, col.astype(np.int64), val, b, n=n)
    with pytest.raises(TypeError):
        P.System(rp, col, val, b.astype(np.float32), n=n)
    # lengths are checked before any pointer crosses the ABI
    with pytest.raises(ValueError):
        P.System(rp, col[:-1], val, b, n=n)
    with pytest.raises(ValueError):
        P.System(rp, col, val[:-3], b, n=n)
    with pytest.raises(ValueError):
        P.System(rp, col, val, b[:-1], n=n)
    with pytest.raises(ValueError):
        P.System(rp, col, val, np.concatenate([b, b])[::2], n=n)  # not contiguous


@pytest.mark.parametrize("zeta,phi,expect", [(0.0, 1.0, "INVALID_ARG"), (1.0, -1.0, "INVALID_ARG"),
                                             (float("nan"), 1.0, "INVALID_ARG")])
def test_augmented_validation(zeta, phi, expect):
    rp, col, val, b, n = _good()
    h = C.c_void_p()
    rc = P.lib().asyrk_create_augmented(C.byref(h), rp.size - 1, n, rp.ctypes.data, col.ctypes.data,
                                        val.ctypes.data, P.F32, b.ctypes.data, zeta, phi, P.MEM_HOST, None)
    assert P.STATUS[rc] == expect


def test_augmented_rejects_empty_column():
    rp, col, val, b, n = _good()
    h = C.c_void_p()
    rc = P.lib().asyrk_create_augmented(C.byref(h), rp.size - 1, n + 5, rp.ctypes.data, col.ctypes.data,
                                        val.ctypes.data, P.F32, b.ctypes.data, 0.5, 1.0, P.MEM_HOST, None)
    assert P.STATUS[rc] == "ZERO_ROW"
