"""The allocation-free lambda_max (asyrk_lambda_max_noalloc) against the
allocating one, through the C ABI.

Both run the same power iteration (Section 1 notation: lambda_max(A^T A),
feeding Corollary 1's bound on tau); the scatter z += A^T y uses atomic adds,
whose order varies from run to run, so the two agree to rounding: 1e-12
relative on lambda (a Rayleigh quotient, stationary at the converged vector)
and exactly on Corollary 1's tau.  Two calls in a row, the second on a
smaller system, show that the shared scratch carries nothing over; a system
too large for the scratch is refused.
"""
import ctypes as C

import numpy as np
import pytest

import paper_1401_4780_amd as P
import synth

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _system(m, n, k, seed, dtype="f32"):
    s = synth.uniform_rows(m, n, k, seed=seed, dtype=dtype, require_full_columns=False)
    return P.System(_dev(s.row_ptr), _dev(s.col), _dev(s.val), _dev(s.b), n=s.n, dtype=dtype)


def _call(fn, sysm, iters, seed):
    lam, tau = C.c_double(), C.c_double()
    rc = fn(sysm._h, iters, seed, C.byref(lam), C.byref(tau))
    assert P.STATUS[rc] == "OK", P.STATUS[rc]
    return lam.value, tau.value


def test_noalloc_lambda_max_matches_allocating_entry_point():
    L = P.lib()
    print("[gpu-case] lambda_max noalloc: 400k x 100k then 3000 x 600", flush=True)
    big = _system(400_000, 100_000, 12, seed=41)
    small = _system(3000, 600, 7, seed=42, dtype="f64")
    # two calls in a row on the scratch, the second with the smaller system
    nb = _call(L.asyrk_lambda_max_noalloc, big, 80, 5)
    ns = _call(L.asyrk_lambda_max_noalloc, small, 80, 5)
    ab = _call(L.asyrk_lambda_max, big, 80, 5)
    as_ = _call(L.asyrk_lambda_max, small, 80, 5)
    for (ln, tn), (la, ta) in ((nb, ab), (ns, as_)):
        assert abs(ln - la) <= 1e-12 * la, (ln, la)
        assert tn == ta, (tn, ta)
    # the small system again after the big one: the scratch's old contents do not matter
    ns2 = _call(L.asyrk_lambda_max_noalloc, small, 80, 5)
    assert abs(ns2[0] - as_[0]) <= 1e-12 * as_[0] and ns2[1] == as_[1]
    # the binding's flag reaches the same entry point
    lam, tau = small.lambda_max(iters=80, seed=5, noalloc=True)
    assert abs(lam - as_[0]) <= 1e-12 * as_[0] and tau == as_[1]
    big.close()
    small.close()


def test_noalloc_lambda_max_refuses_a_system_beyond_its_scratch():
    L = P.lib()
    print("[gpu-case] lambda_max noalloc: 8.4M rows refused", flush=True)
    s = _system(8_400_000, 2000, 2, seed=43)
    lam, tau = C.c_double(-1.0), C.c_double(-1.0)
    rc = L.asyrk_lambda_max_noalloc(s._h, 10, 1, C.byref(lam), C.byref(tau))
    assert P.STATUS[rc] == "SCRATCH"
    assert b"64 MiB" in L.asyrk_last_error_message()
    assert lam.value == -1.0 and tau.value == -1.0
    s.close()
