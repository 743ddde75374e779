"""Pins for the oracle's random row selection.

The paper picks row i with probability ||a_i||^2 / ||A||_F^2 (Section 1) or,
in Algorithm 1, with equal probability.  The oracle draws it from a
Philox4x32-10 block (counter = ticket) through a Vose alias table.  These
tests pin each piece to something outside the oracle: the generator's
published known-answer vectors, exact big-integer arithmetic for the bucket,
the exact probabilities the alias table encodes, and chi-square tests.
"""
from pathlib import Path

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = Path(__file__).resolve().parent / "golden"


def _kat_rows():
    rows = []
    for line in (GOLDEN / "philox4x32_10_kat.txt").read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        vals = [int(t, 16) for t in line.split()]
        rows.append((vals[:4], vals[4:6], vals[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert list(oracle.philox4x32_10(ctr, key)) == expect


def test_bucket_and_counter_layout_exact():
    """Ticket j uses counter (j lo, j hi, stream, 0) and key (seed lo, seed hi);
    the bucket is floor(U * m / 2^64) with U = u1*2^32 + u0, checked with
    Python integers (no 64-bit overflow possible)."""
    for m in (1, 2, 3, 1000, 2_000_003, 4_000_000, 2**31 - 1):
        for seed, stream, ticket0 in ((0, 0, 0), (2**40 + 7, 3, 2**33 - 5)):
            rows = oracle.sample_rows(m, seed, 16, ticket0=ticket0, stream=stream)
            for q in range(16):
                j = ticket0 + q
                u = oracle.philox4x32_10([j & 0xFFFFFFFF, j >> 32, stream, 0],
                                         [seed & 0xFFFFFFFF, seed >> 32])
                big = (int(u[1]) << 32) | int(u[0])
                assert rows[q] == (big * m) >> 64


def _reconstruct(thresh, alias):
    """Exact probability of each row under the alias draw (u2 uniform on 2^32)."""
    m = thresh.size
    t = thresh.astype(np.float64) / 2.0**32
    keep = np.where(alias == np.arange(m), 1.0, t)  # a self-aliased bucket always yields itself
    give = 1.0 - keep
    p = keep.copy()
    np.add.at(p, alias, give)
    return p / m


@pytest.mark.parametrize("kind", ["random", "equal", "extreme", "one", "two", "near_unit"])
def test_alias_table_encodes_the_weights(kind):
    rng = np.random.default_rng(11)
    if kind == "random":
        w = rng.exponential(size=997)
    elif kind == "equal":
        w = np.ones(500)
    elif kind == "extreme":
        w = np.concatenate([rng.uniform(1e-9, 1e-6, 300), rng.uniform(1e3, 1e6, 7)])
    elif kind == "one":
        w = np.array([3.5])
    elif kind == "two":
        w = np.array([1.0, 3.0])
    else:  # unit rows rounded to float32: weights within ~1e-7 of 1
        w = 1.0 + rng.normal(scale=1e-7, size=4096)
    thresh, alias = oracle.alias_build(w)
    m = w.size
    assert np.all(thresh <= 2**32)
    assert np.all((alias >= 0) & (alias < m))
    p = _reconstruct(thresh, alias)
    target = w / w.sum()
    # each bucket's threshold is truncated to 2^-32; a row appears in at most
    # (1 + number of buckets aliasing it) buckets; FP64 drift in the Vose
    # bookkeeping is far below that
    deg = 1 + np.bincount(alias, minlength=m)
    assert np.all(np.abs(p - target) <= (deg * 2.0**-32 + 1e-12) / m)


def test_chi_square_norm_weighted():
    rng = np.random.default_rng(3)
    w = rng.exponential(size=64) + 0.05
    thresh, alias = oracle.alias_build(w)
    n_draw = 1_000_000
    rows = oracle.sample_rows(w.size, 12345, n_draw, thresh=thresh, alias=alias)
    counts = np.bincount(rows, minlength=w.size)
    _, pval = stats.chisquare(counts, n_draw * w / w.sum())
    assert pval > 1e-4


def test_chi_square_uniform():
    rows = oracle.sample_rows(97, 77, 500_000)
    counts = np.bincount(rows, minlength=97)
    _, pval = stats.chisquare(counts)
    assert pval > 1e-4


def test_chi_square_coordinate_draw():
    """Algorithm 1 picks t uniformly in supp(a_i): t = floor(u3 * theta / 2^32)."""
    _, u3 = oracle.sample_rows(10, 5, 300_000, with_u3=True)
    theta = 13
    t = (u3.astype(np.uint64) * np.uint64(theta)) >> np.uint64(32)
    counts = np.bincount(t.astype(np.int64), minlength=theta)
    assert counts.size == theta
    _, pval = stats.chisquare(counts)
    assert pval > 1e-4


def test_ticket_ranges_compose_and_streams_differ():
    a = oracle.sample_rows(1000, 9, 300)
    b = oracle.sample_rows(1000, 9, 100, ticket0=200)
    assert np.array_equal(a[200:], b)
    c = oracle.sample_rows(1000, 9, 300, stream=1)
    d = oracle.sample_rows(1000, 10, 300)
    assert (a != c).mean() > 0.9 and (a != d).mean() > 0.9
