"""Pins for the oracle's Kaczmarz update, run loop and delay model.

Each test checks the oracle against something the paper or plain mathematics
fixes, never against a retyped copy of its own formula:

* closed forms: a one-row system; rows that are scaled unit vectors;
* the two per-step identities of eq. (2) (projection onto the hyperplane and
  the Pythagorean decrease, Section 1) which together determine the step;
* the exact one-step expectation of Section 1, by enumerating every row;
* the expected linear rate of Section 1 and of Corollary 1, over many seeds;
* the limit point: the least-squares (minimum-norm) solution;
* brute force with explicit iterate snapshots for the read delay of eq. (3).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth


def _tiny(m, n, k, seed, normalize=True):
    return synth.uniform_rows(m, n, k, seed, dtype="f64", normalize=normalize,
                              require_full_columns=False)


def _run(s, x0, gamma, nsteps, seed, **kw):
    return oracle.rk_run(s.row_ptr, s.col, s.val64, s.b, s.n, x0, gamma, nsteps, seed, **kw)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("gamma", [1.0, 0.5, 1.9])
def test_one_row_closed_form(gamma):
    a = np.array([0.0, 3.0, 0.0, -4.0, 1.0])
    row_ptr = np.array([0, 3])
    col = np.array([1, 3, 4])
    val = a[col]
    b = np.array([2.5])
    x0 = np.array([1.0, -2.0, 0.5, 0.25, 3.0])
    out = oracle.rk_run(row_ptr, col, val, b, 5, x0, gamma, 1, 0)
    expect = x0 - gamma * (a @ x0 - b[0]) / (a @ a) * a
    np.testing.assert_allclose(out["x"], expect, rtol=0, atol=1e-15)


def test_scaled_unit_rows_reach_solution_exactly():
    """Row i is c_i * e_{pi(i)} with c_i a power of two: with gamma = 1 every
    coordinate is exact once its row has been drawn."""
    rng = np.random.default_rng(0)
    n = 40
    perm = rng.permutation(n)
    c = rng.choice([1.0, -1.0, 2.0, -0.5, 4.0], size=n)
    x_star = rng.standard_normal(n)
    row_ptr = np.arange(n + 1)
    b = c * x_star[perm]
    out = oracle.rk_run(row_ptr, perm.astype(np.int32), c, b, n, np.zeros(n), 1.0, 2000, 3,
                        want_rows=True)
    assert np.unique(out["rows"]).size == n
    assert np.array_equal(out["x"], x_star)


# --------------------------------------------------- per-step identities (eq. 2)

@pytest.mark.parametrize("gamma", [1.0, 0.5, 1.7])
def test_per_step_projection_and_pythagoras(gamma):
    s = _tiny(30, 12, 4, seed=5, normalize=False)
    A = s.dense()
    rows = oracle.sample_rows(s.m, 1, 200)
    x = np.random.default_rng(2).standard_normal(s.n)
    for i in rows:
        x1 = oracle.apply_rows(s.row_ptr, s.col, s.val64, s.b, x, gamma, [i])
        a = A[i]
        r0 = a @ x - s.b[i]
        # (a) the new residual of row i is (1 - gamma) times the old one
        assert abs((a @ x1 - s.b[i]) - (1 - gamma) * r0) <= 1e-12 * (1 + abs(r0))
        # (b) the step is along a_i (zero off its support, proportional on it)
        d = x1 - x
        coef = (d @ a) / (a @ a)
        np.testing.assert_allclose(d, coef * a, atol=1e-13 * (1 + np.abs(d).max()))
        # (c) Pythagorean decrease of the error
        e0 = np.sum((x - s.x_star) ** 2)
        e1 = np.sum((x1 - s.x_star) ** 2)
        assert abs(e1 - (e0 - gamma * (2 - gamma) * r0 * r0 / (a @ a))) <= 1e-11 * (1 + e0)
        x = x1


def test_run_equals_enumerated_rows():
    s = _tiny(50, 20, 5, seed=6, normalize=False)
    w = (s.dense() ** 2).sum(axis=1)
    thresh, alias = oracle.alias_build(oracle.row_weights(s.row_ptr, s.val64))
    rows = oracle.sample_rows(s.m, 42, 500, thresh=thresh, alias=alias)
    out = _run(s, np.zeros(s.n), 0.8, 500, 42, want_rows=True)
    assert np.array_equal(out["rows"], rows)
    x = oracle.apply_rows(s.row_ptr, s.col, s.val64, s.b, np.zeros(s.n), 0.8, rows)
    assert np.array_equal(out["x"], x)
    np.testing.assert_allclose(oracle.row_weights(s.row_ptr, s.val64), w, rtol=1e-14)


# ----------------------------------------------------- exact one-step expectation

@pytest.mark.parametrize("gamma", [1.0, 0.6])
def test_exact_expectation_all_coordinates(gamma):
    """E_i ||x+ - x*||^2 = ||x - x*||^2 - gamma(2-gamma) ||Ax-b||^2 / ||A||_F^2
    with P(i) = ||a_i||^2/||A||_F^2 (Section 1, with step length gamma)."""
    s = _tiny(25, 10, 4, seed=8, normalize=False)
    A = s.dense()
    w = (A ** 2).sum(axis=1)
    fro2 = w.sum()
    x = np.random.default_rng(1).standard_normal(s.n)
    e = np.empty(s.m)
    for i in range(s.m):
        xi = oracle.apply_rows(s.row_ptr, s.col, s.val64, s.b, x, gamma, [i])
        e[i] = np.sum((xi - s.x_star) ** 2)
    lhs = np.sum(w / fro2 * e)
    rhs = np.sum((x - s.x_star) ** 2) - gamma * (2 - gamma) * np.sum((A @ x - s.b) ** 2) / fro2
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_exact_expectation_single_coordinate():
    """Algorithm 1 (i uniform, t uniform in supp a_i, step gamma*theta_i):
    E ||x+ - x*||^2 = ||x - x*||^2 - (1/m) sum_i (2 gamma - gamma^2 theta_i) r_i^2 / ||a_i||^2."""
    s = _tiny(20, 9, 4, seed=9, normalize=False)
    A = s.dense()
    gamma = 0.2
    x = np.random.default_rng(4).standard_normal(s.n)
    acc = 0.0
    for i in range(s.m):
        th = int(s.row_ptr[i + 1] - s.row_ptr[i])
        for t in range(th):
            xi = oracle.apply_rows(s.row_ptr, s.col, s.val64, s.b, x, gamma, [i], coords=[t])
            acc += np.sum((xi - s.x_star) ** 2) / th
    lhs = acc / s.m
    r = A @ x - s.b
    w = (A ** 2).sum(axis=1)
    theta = np.diff(s.row_ptr)
    rhs = np.sum((x - s.x_star) ** 2) - np.sum((2 * gamma - gamma**2 * theta) * r * r / w) / s.m
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_single_coordinate_run_equals_enumeration():
    s = _tiny(40, 15, 5, seed=10)
    rows, u3 = oracle.sample_rows(s.m, 7, 300, with_u3=True)
    theta = np.diff(s.row_ptr)[rows]
    t = ((u3.astype(np.uint64) * theta.astype(np.uint64)) >> np.uint64(32)).astype(np.int32)
    out = _run(s, np.zeros(s.n), 0.2, 300, 7, uniform=True, update_one=True, want_rows=True)
    assert np.array_equal(out["rows"], rows)
    x = oracle.apply_rows(s.row_ptr, s.col, s.val64, s.b, np.zeros(s.n), 0.2, rows, coords=t)
    assert np.array_equal(out["x"], x)


# ------------------------------------------------------------- expected rates

def _lambda_min_nonzero(A):
    ev = np.linalg.eigvalsh(A.T @ A)
    return ev[ev > 1e-10 * ev.max()].min()


@pytest.mark.parametrize("gamma", [1.0, 0.5])
def test_expected_rate_bound_rk(gamma):
    """E||x_K - x*||^2 <= (1 - gamma(2-gamma) lambda_min/||A||_F^2)^K ||x_0 - x*||^2."""
    s = _tiny(60, 20, 5, seed=12)
    A = s.dense()
    lam = _lambda_min_nonzero(A)
    fro2 = (A ** 2).sum()
    K = 120
    e0 = np.sum(s.x_star ** 2)
    ratios = [np.sum((_run(s, np.zeros(s.n), gamma, K, seed)["x"] - s.x_star) ** 2) / e0
              for seed in range(300)]
    bound = (1 - gamma * (2 - gamma) * lam / fro2) ** K
    assert bound < 0.5
    assert np.mean(ratios) <= bound


def test_corollary_rate_single_coordinate():
    """Corollary 1 with tau = 0 (gamma = 1/psi = 1/mu, unit rows, uniform rows):
    E||x_j - x*||^2 <= (1 - lambda_min / (m (mu + 1)))^j ||x_0 - x*||^2."""
    s = _tiny(60, 20, 5, seed=13)
    A = s.dense()
    lam = _lambda_min_nonzero(A)
    lam_max = np.linalg.eigvalsh(A.T @ A).max()
    assert 2 * np.e * lam_max * 1 / s.m <= 1.0  # the corollary's condition at tau = 0
    mu = int(np.diff(s.row_ptr).max())
    K = 600
    e0 = np.sum(s.x_star ** 2)
    ratios = [np.sum((_run(s, np.zeros(s.n), 1.0 / mu, K, seed, uniform=True,
                           update_one=True)["x"] - s.x_star) ** 2) / e0 for seed in range(200)]
    bound = (1 - lam / (s.m * (mu + 1))) ** K
    assert bound < 0.8
    assert np.mean(ratios) <= bound


# ---------------------------------------------------------------- limit point

def test_limit_is_least_squares_solution_full_rank():
    """m=2000, n=500, 10 nonzeros per row (the small FP64 configuration)."""
    s = synth.uniform_rows(2000, 500, 10, seed=0, dtype="f64")
    A = s.dense()
    ls = np.linalg.lstsq(A, s.b, rcond=None)[0]
    assert np.linalg.norm(ls - s.x_star) <= 1e-12 * np.linalg.norm(s.x_star)
    out = _run(s, np.zeros(s.n), 1.0, 200 * s.m, 0, curve_every=s.m, x_ref=ls)
    assert out["err"][-1] <= 1e-12
    # the error contracts every sweep until it reaches rounding level, and
    # after 20 sweeps it is inside the expected-rate bound exp(-20 lambda_min / 2)
    err = out["err"]
    big = err[:-1] > 1e-13
    assert np.all(err[1:][big] < err[:-1][big])
    lam = _lambda_min_nonzero(A)
    assert err[20] <= np.exp(-20 * lam / 2)


def test_limit_is_minimum_norm_solution_underdetermined():
    """m < n as in the paper's experiments: from x0 = 0 the iterates stay in
    range(A^T) and reach the minimum-norm solution pinv(A) b."""
    s = _tiny(80, 100, 6, seed=14)
    A = s.dense()
    xmn = np.linalg.pinv(A) @ s.b
    out = _run(s, np.zeros(s.n), 1.0, 3000 * s.m, 1)
    np.testing.assert_allclose(out["x"], xmn, atol=1e-9 * np.linalg.norm(xmn))
    assert np.linalg.norm(A @ out["x"] - s.b) <= 1e-9 * np.linalg.norm(s.b)


def test_residual_matches_sparse_product():
    s = _tiny(300, 100, 7, seed=15, normalize=False)
    x = np.random.default_rng(0).standard_normal(s.n)
    M = sp.csr_matrix((s.val64, s.col, s.row_ptr), shape=(s.m, s.n))
    n2, r = oracle.residual(s.row_ptr, s.col, s.val64, s.b, x, want_r=True)
    np.testing.assert_allclose(r, s.b - M @ x, rtol=1e-13, atol=1e-13)
    assert abs(n2 - np.sum((s.b - M @ x) ** 2)) <= 1e-12 * n2


# ------------------------------------------------------------------ delay (eq. 3)

def _delay_bruteforce(s, gamma, rows, tau, update_coords=None):
    A = s.dense()
    w = (A ** 2).sum(axis=1)
    xs = [np.zeros(s.n)]
    for j, i in enumerate(rows):
        xr = xs[max(0, j - tau)]
        r = A[i] @ xr - s.b[i]
        x = xs[-1].copy()
        x -= gamma * r / w[i] * A[i]
        xs.append(x)
    return xs[-1]


@pytest.mark.parametrize("tau", [1, 3, 7, 50])
def test_delay_model_bruteforce(tau):
    """Ticket j reads x_{j - tau} and updates x_j (eq. (3) with k(j) = j - tau)."""
    s = _tiny(40, 16, 4, seed=16)
    K = 400
    out = _run(s, np.zeros(s.n), 0.7, K, 3, tau=tau, want_rows=True)
    ref = _delay_bruteforce(s, 0.7, out["rows"], tau)
    np.testing.assert_allclose(out["x"], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_delay_zero_is_plain_rk_bitwise():
    s = _tiny(40, 16, 4, seed=17)
    a = _run(s, np.zeros(s.n), 1.0, 500, 2)["x"]
    b = _run(s, np.zeros(s.n), 1.0, 500, 2, tau=0)["x"]
    assert np.array_equal(a, b)


def test_delay_slows_but_small_delay_still_converges():
    s = _tiny(400, 100, 5, seed=18)
    e = [_run(s, np.zeros(s.n), 1.0, 30 * s.m, 4, tau=tau, curve_every=s.m,
              x_ref=s.x_star)["err"][-1] for tau in (0, 4, 16)]
    assert e[0] < 1e-6 and e[1] < 1e-4 and e[2] < 1e-2
