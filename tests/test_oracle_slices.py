"""Pins for the oracle's slice scheme (the paper's experiments: equal row
slices per thread, each visited in order and reshuffled after every scan).

The row order is a keyed permutation; what the paper fixes, and these tests
check, is that every sweep visits every row exactly once, that each worker
stays inside its own slice, that the order changes from sweep to sweep, and
that the method still converges to the least-squares solution."""
import numpy as np
import pytest
from scipy import stats

import oracle
import synth


@pytest.mark.parametrize("m,R", [(1, 1), (2, 1), (10, 3), (997, 1), (1000, 7), (4096, 64), (5000, 4999),
                                 (300, 1000)])
def test_each_sweep_is_a_permutation_respecting_slices(m, R):
    L = -(-m // R)
    for sweep in (0, 1, 2**33 + 5):
        order = oracle.slice_order(m, R, 12345, sweep)
        assert np.array_equal(np.sort(order), np.arange(m))
        # round-robin over workers: the q-th visit of the sweep belongs to the
        # worker whose slice holds it, and positions advance worker by worker
        owners = order // L
        live = [w for w in range(R) if w * L < m]
        lens = [min(L, m - w * L) for w in live]
        expect = [w for k in range(L) for w, ln in zip(live, lens) if k < ln]
        assert np.array_equal(owners, expect)


def test_order_changes_between_sweeps_and_seeds():
    a = oracle.slice_order(1000, 1, 1, 0)
    b = oracle.slice_order(1000, 1, 1, 1)
    c = oracle.slice_order(1000, 1, 2, 0)
    assert (a != b).mean() > 0.9 and (a != c).mean() > 0.9


def test_positions_are_spread_uniformly():
    m = 64
    pos = np.array([np.nonzero(oracle.slice_order(m, 1, 7, s) == 0)[0][0] for s in range(6400)])
    _, pval = stats.chisquare(np.bincount(pos, minlength=m))
    assert pval > 1e-4


def test_slice_run_equals_its_row_sequence_and_converges():
    s = synth.uniform_rows(2000, 500, 10, seed=0, dtype="f64")
    run = oracle.rk_run(s.row_ptr, s.col, s.val64, s.b, s.n, np.zeros(s.n), 1.0, 3 * s.m, 9,
                        slices=True, workers=16, want_rows=True)
    rows = run["rows"]
    for k in range(3):
        assert np.array_equal(rows[k * s.m:(k + 1) * s.m], oracle.slice_order(s.m, 16, 9, k))
    x = oracle.apply_rows(s.row_ptr, s.col, s.val64, s.b, np.zeros(s.n), 1.0, rows)
    assert np.array_equal(run["x"], x)
    ls = np.linalg.lstsq(s.dense(), s.b, rcond=None)[0]
    out = oracle.rk_run(s.row_ptr, s.col, s.val64, s.b, s.n, np.zeros(s.n), 1.0, 120 * s.m, 9,
                        slices=True, workers=1, curve_every=s.m, x_ref=ls)
    assert out["err"][-1] <= 1e-12
    # without replacement is not slower per sweep here (the paper reports it faster)
    rep = oracle.rk_run(s.row_ptr, s.col, s.val64, s.b, s.n, np.zeros(s.n), 1.0, 10 * s.m, 9,
                        curve_every=s.m, x_ref=ls)
    assert out["err"][10] <= 1.5 * rep["err"][10]
