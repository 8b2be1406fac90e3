"""Pins of the oracle's Gaussian test matrix against published definitions
(Philox4x32-10 known answers, the elementary functions it replaces, and the normal
distribution).  CPU only."""
import math

import numpy as np
import pytest
import scipy.stats

from conftest import read_golden
from oracle import rng


def test_philox_known_answers():
    rows = read_golden("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for r in rows:
        vals = [int(x, 16) for x in r]
        ctr, key, want = vals[:4], vals[4:6], vals[6:]
        got = rng.philox4x32_10(*[np.uint64(c) for c in ctr], *[np.uint64(k) for k in key])
        assert [int(g) for g in got] == want


def test_uniform52_range_and_endpoints():
    lo = rng.uniform52(np.uint64(0), np.uint64(0))
    hi = rng.uniform52(np.uint64(0xFFFFFFFF), np.uint64(0xFFFFFFFF))
    assert lo == 2.0 ** -53
    assert hi == 1.0 - 2.0 ** -53


@pytest.mark.parametrize("seed", [1, 7])
def test_own_log_matches_libm(seed):
    g = np.random.default_rng(seed)
    x = np.concatenate([g.random(20000), 2.0 ** -g.integers(1, 53, 2000) * (1 + g.random(2000)),
                        [2.0 ** -53, 1.0 - 2.0 ** -53, 0.5, rng.SQRT_HALF]])
    x = x[(x > 0) & (x < 1)]
    got = rng.own_log(x)
    ref = np.array([math.log(v) for v in x])
    # within 4 ulp relative (the series and the final e ln2 + ln m each round)
    assert np.all(np.abs(got - ref) <= 8.9e-16 * np.abs(ref) + 1e-19)


def test_own_sqrt_matches_libm():
    g = np.random.default_rng(3)
    y = np.concatenate([g.random(20000) * 80.0, 10.0 ** g.uniform(-17, 2, 5000), [1.0, 4.0, 2.0]])
    y = y[y > 0]
    got = rng.own_sqrt(y)
    ref = np.sqrt(y)
    assert np.all(np.abs(got - ref) <= 2.3e-16 * ref)


def test_own_sincos_matches_libm():
    g = np.random.default_rng(4)
    u = np.concatenate([g.random(50000), [0.125, 0.25, 0.375, 0.5, 0.75, 2.0 ** -53, 1 - 2.0 ** -53]])
    s, c = rng.own_sincos_2pi(u)
    th = 2.0 * math.pi * u
    assert np.max(np.abs(s - np.sin(th))) < 1e-15
    assert np.max(np.abs(c - np.cos(th))) < 1e-15
    assert np.max(np.abs(s * s + c * c - 1.0)) < 1e-15


def test_gaussian_statistics():
    G = rng.gaussian_matrix(0x1234, 400, 250)
    x = G.ravel()
    assert abs(x.mean()) < 4.0 / math.sqrt(x.size)
    assert abs(x.var() - 1.0) < 6.0 * math.sqrt(2.0 / x.size)
    assert scipy.stats.kstest(x, "norm").pvalue > 1e-3
    # the two members of a Box-Muller pair are uncorrelated
    c = np.corrcoef(G[:, 0::2].ravel(), G[:, 1::2].ravel())[0, 1]
    assert abs(c) < 5.0 / math.sqrt(G.size / 2)
    # fourth moment of a standard normal is 3
    assert abs(np.mean(x ** 4) - 3.0) < 0.1


def test_gaussian_slicing_and_streams():
    full = rng.gaussian_matrix(99, 37, 23)
    assert np.array_equal(rng.gaussian_matrix(99, 10, 7, row0=5, col0=3), full[5:15, 3:10])
    assert np.array_equal(rng.gaussian_matrix(99, 37, 1, col0=22), full[:, 22:23])
    other = rng.gaussian_matrix(99, 37, 23, stream=1)
    assert not np.any(other == full)
    other_b = rng.gaussian_matrix(99, 37, 23, batch=1)
    assert not np.any(other_b == full)
    assert rng.gaussian_matrix(99, 0, 5).shape == (0, 5)
