"""Sanity checks of the seeded input generator (not of the method).

The paper's recipe: random nonzero positions, N(0,1) values, rows normalized
(Section "Experiments"); with normalized rows ||A||_F^2 = m (Section 1), and
lambda_max <= mu * nu for sparse A (Section 1, notation).
"""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_uniform_rows_structure(dtype):
    s = synth.uniform_rows(2000, 500, 10, seed=0, dtype=dtype)
    assert s.row_ptr[0] == 0 and s.row_ptr[-1] == 20000
    assert np.all(np.diff(s.row_ptr) == 10)
    c = s.col.reshape(2000, 10)
    assert np.all(np.diff(c, axis=1) > 0)
    assert c.min() >= 0 and c.max() < 500
    assert np.bincount(s.col, minlength=500).min() > 0
    w = np.add.reduceat(s.val64 ** 2, s.row_ptr[:-1])
    tol = {"f64": 1e-15, "f32": 1e-6, "bf16": 2e-2}[dtype]
    np.testing.assert_allclose(w, 1.0, atol=tol)
    if dtype == "f64":
        assert abs(w.sum() - s.m) <= 1e-10  # ||A||_F^2 = m
    # b = A x* in float64 from the stored values
    A = s.dense()
    np.testing.assert_allclose(A @ s.x_star, s.b, rtol=1e-13, atol=1e-13)


def test_lambda_max_bound():
    s = synth.uniform_rows(300, 100, 6, seed=3, dtype="f64")
    A = s.dense()
    lam_max = np.linalg.eigvalsh(A.T @ A).max()
    mu = np.diff(s.row_ptr).max()
    nu = np.bincount(s.col, minlength=s.n).max()
    assert lam_max <= mu * nu
    # the Gaussian-ensemble estimate (1 + sqrt(n/m))^2 m/n is the right scale
    est = (1 + np.sqrt(s.n / s.m)) ** 2 * s.m / s.n
    assert 0.5 * est < lam_max < 1.5 * est


def test_determinism_and_seed_sensitivity():
    a = synth.uniform_rows(500, 200, 8, seed=7, dtype="f32")
    b = synth.uniform_rows(500, 200, 8, seed=7, dtype="f32")
    c = synth.uniform_rows(500, 200, 8, seed=8, dtype="f32")
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    assert np.array_equal(a.b, b.b)
    assert not np.array_equal(a.col, c.col)


def test_bf16_rounding_is_nearest_even():
    f = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, 1.0 + 2**-9, -2.5, 1.0 + 2**-7 + 2**-9],
                 dtype=np.float32)
    back = synth.f64_from_bf16_bits(synth.bf16_bits_from_f32(f))
    np.testing.assert_array_equal(back, [1.0, 1.0, 1.0 + 2**-6, 1.0, -2.5, 1.0 + 2**-7 + 2**-8 * 0])


def test_skewed_rows_shape():
    s = synth.skewed_rows(20000, 5000, seed=2)
    lens = np.diff(s.row_ptr)
    assert lens.min() >= 4 and lens.max() <= 2000
    assert 20 < lens.mean() < 33
    for i in range(0, s.m, 997):
        c = s.col[s.row_ptr[i]:s.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    counts = np.bincount(s.col, minlength=s.n)
    assert counts.max() > 0.5 * s.m  # one hot column sits in most rows
    # x* lies in range(A^T): b = A x* is consistent and nonzero
    assert np.linalg.norm(s.b) > 0
    assert abs(np.sqrt(np.mean(s.x_star ** 2)) - 1.0) < 1e-12


def test_serving_stream():
    specs = synth.serving_specs(200, seed=4)
    assert specs[:, 0].min() >= 1000 and specs[:, 0].max() <= 200000
    assert np.all(specs[:, 1] == specs[:, 0] // 4)
    s = synth.serving_system(3, 1500, 375)
    lens = np.diff(s.row_ptr)
    assert lens.min() >= 8 and lens.max() <= 64
    t = synth.poisson_arrivals(1000, 50.0)
    assert np.all(np.diff(t) > 0) and 10 < t[-1] < 30


def test_as_dtype_equals_direct_generation():
    a = synth.uniform_rows(700, 200, 6, seed=9, dtype="f64")
    for dt in ("f32", "bf16"):
        b = synth.as_dtype(a, dt)
        c = synth.uniform_rows(700, 200, 6, seed=9, dtype=dt)
        assert np.array_equal(b.col, c.col) and np.array_equal(b.val, c.val)
        assert np.array_equal(b.b, c.b) and np.array_equal(b.x_star, c.x_star)
