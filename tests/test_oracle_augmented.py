"""Pins for the inconsistent-system extension (paper, Section "Extension to
Inconsistent Systems"): the augmented matrix, its smallest nonzero singular
value and Frobenius norm in closed form, the optimal (zeta, phi), and RK on
the augmented system reaching the least-squares solution."""
import numpy as np
import pytest

import oracle
import synth


def _inconsistent(m=60, n=20, k=5, seed=3):
    s = synth.uniform_rows(m, n, k, seed=seed, dtype="f64", require_full_columns=True)
    b = s.b + 0.3 * np.random.default_rng(seed).standard_normal(m)  # not in range(A)
    return s, b


def test_augmented_matrix_blocks():
    s, b = _inconsistent()
    rp, col, val, ba = oracle.augmented_system(s.row_ptr, s.col, s.val64, b, s.n, 0.7, 1.3)
    N = s.n + s.m
    M = np.zeros((N, N))
    M[np.repeat(np.arange(N), np.diff(rp)), col] = val
    A = s.dense()
    assert np.allclose(M[:s.n, :s.n], 0) and np.allclose(M[:s.n, s.n:], 1.3 * A.T)
    assert np.allclose(M[s.n:, :s.n], A) and np.allclose(M[s.n:, s.n:], -0.7 * np.eye(s.m))
    assert np.allclose(ba, np.concatenate([1.3 * A.T @ b, np.zeros(s.m)]))


# The closed form treats each 2x2 block [[0, phi s], [s, -zeta]] through its
# eigenvalues; they are its singular values only when the block is symmetric,
# i.e. phi = 1 (the value the paper ends up recommending).  The Frobenius norm
# holds for every phi.
@pytest.mark.parametrize("zeta,phi", [(0.3, 1.0), (1.7, 1.0), (0.55, 1.0), (0.05, 3.0)])
def test_min_singular_value_and_frobenius_closed_forms(zeta, phi):
    s, b = _inconsistent()
    A = s.dense()
    sig = np.linalg.svd(A, compute_uv=False)
    sr = sig[sig > 1e-12].min()
    rp, col, val, _ = oracle.augmented_system(s.row_ptr, s.col, s.val64, b, s.n, zeta, phi)
    N = s.n + s.m
    M = np.zeros((N, N))
    M[np.repeat(np.arange(N), np.diff(rp)), col] = val
    sv = np.linalg.svd(M, compute_uv=False)
    smin = sv[sv > 1e-10].min()
    expect = min(zeta, -zeta / 2 + 0.5 * np.sqrt(zeta**2 + 4 * phi * sr**2))
    assert abs(smin - expect) <= 1e-10 * expect
    fro2 = (1 + phi**2) * np.sum(A**2) + s.m * zeta**2
    assert abs(np.sum(M**2) - fro2) <= 1e-10 * fro2


def test_optimal_zeta_phi():
    """sigma_min(M)^2 / ||M||_F^2 is largest at zeta = sigma_r sqrt(phi/2), phi = 1."""
    s, b = _inconsistent()
    A = s.dense()
    sr = np.linalg.svd(A, compute_uv=False).min()

    def ratio(z, p):
        rp, col, val, _ = oracle.augmented_system(s.row_ptr, s.col, s.val64, b, s.n, z, p)
        N = s.n + s.m
        M = np.zeros((N, N))
        M[np.repeat(np.arange(N), np.diff(rp)), col] = val
        sv = np.linalg.svd(M, compute_uv=False)
        return sv[sv > 1e-10].min() ** 2 / np.sum(M**2)

    best = ratio(sr / np.sqrt(2), 1.0)
    fro2 = np.sum(A**2)
    assert abs(best - sr**2 / (4 * fro2 + s.m * sr**2)) <= 1e-9 * best
    for z in np.linspace(0.2, 3.0, 9) * sr / np.sqrt(2):
        for p in (0.5, 0.8, 1.25, 2.0):
            assert ratio(z, p) <= best * (1 + 1e-9)


def test_rk_on_augmented_system_reaches_least_squares():
    s, b = _inconsistent()
    A = s.dense()
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.linalg.norm(A @ x_ls - b) > 1e-2 * np.linalg.norm(b)  # truly inconsistent
    sr = np.linalg.svd(A, compute_uv=False).min()
    zeta = sr / np.sqrt(2)
    rp, col, val, ba = oracle.augmented_system(s.row_ptr, s.col, s.val64, b, s.n, zeta, 1.0)
    N = s.n + s.m
    out = oracle.rk_run(rp, col, val, ba, N, np.zeros(N), 1.0, 4000 * N, 2)
    x = out["x"][:s.n] / zeta
    assert np.linalg.norm(x - x_ls) <= 1e-9 * np.linalg.norm(x_ls)
