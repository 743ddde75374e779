"""The delay simulator swept across Corollary 1's condition on tau (CPU only).

The oracle's delayed run evaluates ticket j against x_{j - tau} and applies it
to x_j: the worst case of eq. (3), k(j) = j - tau, for every ticket.  On a
system whose Corollary 1 bound tau_max = floor(||A||_F^2 / (2 e lambda_max)) - 1
is about 20:

* single-coordinate updates (Algorithm 1, uniform rows, gamma = 1/psi): for
  every tau up to tau_max, psi <= mu + 1 and the seed-averaged squared error
  after K sweeps is below the corollary's rate (1 - lambda_min / (m (mu + 1)))^j;
  the per-sweep contraction stays within a band of the tau = 0 one;
* beyond the bound (gamma held at 1/(mu + 1)) the contraction weakens as tau
  grows and the iteration diverges far above it;
* all-coordinate updates (gamma = 1, the experiments' variant): within the
  band up to tau_max, measurably slower a few times above it and divergent
  further up, at a smaller multiple of tau_max than single-coordinate updates
  (a full-row update acts like about nnz single-coordinate ones, the paper's
  remark on density in Section "Experiments").

Reading of Corollary 1 used here: its proof bounds rho^(tau+1) by e through
(1 + 2 e lambda_max / m)^(m / (2 e lambda_max)) <= e, i.e. with
rho = 1 + 2 e lambda_max / m; with that rho all three step bounds of Theorem 1
hold for gamma = 1/psi inside the condition.  The printed definition carries an
extra factor (tau + 1) in rho - 1, under which rho^tau is not bounded by e and
gamma = 1/psi collapses (about 1e-6 at tau = tau_max on this system).
"""
import math

import numpy as np
import pytest

import oracle
import synth

M, N, K_NNZ = 1200, 300, 5
SWEEPS = 30


@pytest.fixture(scope="module")
def system():
    s = synth.uniform_rows(M, N, K_NNZ, seed=31, dtype="f64")
    A = s.dense()
    ev = np.linalg.eigvalsh(A.T @ A)
    lmax = float(ev[-1])
    lmin = float(ev[ev > 1e-10 * lmax].min())
    fro2 = float((A ** 2).sum())
    tau_max = math.floor(fro2 / (2 * math.e * lmax)) - 1
    return s, lmax, lmin, fro2, tau_max


def _psi(tau, lmax, mu):
    """psi of Theorem 1 with Corollary 1's rho (the proof's reading, see above)."""
    rho = 1.0 + 2.0 * math.e * lmax / M
    return mu + 2.0 * lmax * tau * rho ** tau / M


def _mean_ratio(s, tau, gamma, one, sweeps, seeds):
    """Seed average of ||x_K - x*||^2 / ||x_0 - x*||^2 from x_0 = 0."""
    e0 = float(np.sum(s.x_star ** 2))
    r = []
    for seed in range(seeds):
        out = oracle.rk_run(s.row_ptr, s.col, s.val64, s.b, s.n, np.zeros(s.n), gamma, sweeps * s.m, seed,
                            uniform=one, update_one=one, tau=tau, want_res=False)
        r.append(float(np.sum((out["x"] - s.x_star) ** 2)) / e0)
    return float(np.mean(r))


def _contraction(ratio, sweeps):
    """Mean log decrease of the squared error per sweep (negative: converging)."""
    return math.log(ratio) / sweeps if ratio > 0 and math.isfinite(ratio) else math.inf


def test_system_has_a_moderate_bound(system):
    s, lmax, lmin, fro2, tau_max = system
    assert abs(fro2 - M) < 1e-9 * M  # unit rows: ||A||_F^2 = m (Assumption 1)
    assert 10 <= tau_max <= 40, tau_max
    assert 2 * math.e * lmax * (tau_max + 1) / fro2 <= 1 < 2 * math.e * lmax * (tau_max + 2) / fro2


def test_single_coordinate_inside_the_bound_keeps_the_rate(system):
    s, lmax, lmin, fro2, tau_max = system
    mu = K_NNZ
    rate = (1.0 - lmin / (M * (mu + 1))) ** (SWEEPS * M)
    c = {}
    for tau in (0, tau_max // 2, tau_max):
        psi = _psi(tau, lmax, mu)
        assert psi <= mu + 1, (tau, psi)  # the corollary's bound on psi
        ratio = _mean_ratio(s, tau, 1.0 / psi, True, SWEEPS, 30)
        assert ratio <= rate, (tau, ratio, rate)  # Corollary 1's expected rate
        c[tau] = _contraction(ratio, SWEEPS)
    for tau in (tau_max // 2, tau_max):
        assert c[tau] <= 0.85 * c[0], c  # within 15% of the undelayed contraction


def test_single_coordinate_degrades_beyond_the_bound(system):
    s, lmax, lmin, fro2, tau_max = system
    gamma = 1.0 / (K_NNZ + 1)  # the smallest step Corollary 1 prescribes inside its condition
    c = {mult: _contraction(_mean_ratio(s, mult * tau_max, gamma, True, SWEEPS, 20), SWEEPS)
         for mult in (0, 1, 16, 64)}
    assert c[1] <= 0.98 * c[0] < 0, c  # at the bound: unchanged
    assert c[16] > c[1], c             # far above: weaker contraction
    assert c[64] > 0, c                # further up: the error grows


def test_all_coordinate_inside_band_then_degrades(system):
    s, lmax, lmin, fro2, tau_max = system
    sweeps = 10
    c = {mult: _contraction(_mean_ratio(s, int(mult * tau_max), 1.0, False, sweeps, 20), sweeps)
         for mult in (0, 0.5, 1, 4, 16)}
    assert c[0] < 0
    for mult in (0.5, 1):
        assert c[mult] <= 0.95 * c[0], c  # within 5% below the bound
    assert c[4] > 0.85 * c[0], c          # a few times above: measurably slower
    assert c[16] > 0, c                   # far above: diverges
