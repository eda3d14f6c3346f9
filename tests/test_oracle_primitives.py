"""Pins of the oracle's deterministic primitives against independent references.

Philox4x64-10 against numpy's independent implementation; the project-written
log and sin/cos against mpmath at high precision; the samplers against their
target distributions (scipy.stats) and exact structural properties.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import stats

import oracle


def ulp_err(got, ref_mp):
    ref = float(ref_mp)
    u = math.ulp(ref) if ref != 0 else math.ulp(0.0)
    return abs(float(mpmath.mpf(got) - ref_mp)) / u


def test_philox_matches_numpy():
    rng = np.random.default_rng(123)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(1, 2**63, size=4, dtype=np.int64)]
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        # numpy increments its counter (word 0 first) before generating a block
        bg = np.random.Philox(counter=[ctr[0] - 1, ctr[1], ctr[2], ctr[3]], key=key)
        assert oracle.philox(ctr, key) == [int(x) for x in bg.random_raw(4)]


def test_philox_counter_words_are_independent_streams():
    a = oracle.philox([5, 0, 0, 0], [1, 1])
    assert a != oracle.philox([5, 1, 0, 0], [1, 1])
    assert a != oracle.philox([5, 0, 1, 0], [1, 1])
    assert a != oracle.philox([5, 0, 0, 1], [1, 1])
    assert a != oracle.philox([5, 0, 0, 0], [1, 2])


def test_dlog_accuracy_against_mpmath():
    mpmath.mp.dps = 40
    rng = np.random.default_rng(7)
    xs = np.concatenate([rng.random(3000), np.exp(rng.uniform(-700, 700, 3000)),
                         1.0 + rng.uniform(-1e-3, 1e-3, 1000), [5e-324, 1e-310, 2.2250738585072014e-308]])
    ys = oracle.dlog(xs)
    worst = max(ulp_err(y, mpmath.log(mpmath.mpf(float(x)))) for x, y in zip(xs, ys))
    assert worst <= 3.0, worst  # series form: about 2.6 ulp just above x = 1
    assert oracle.dlog(np.array([1.0]))[0] == 0.0
    for k in (-1000, -3, -1, 1, 2, 10, 1000):
        y = oracle.dlog(np.array([2.0 ** k]))[0]
        assert ulp_err(y, k * mpmath.log(2)) <= 1.0
    special = oracle.dlog(np.array([0.0, -1.0, np.inf]))
    assert special[0] == -np.inf and np.isnan(special[1]) and special[2] == np.inf


def test_dsincos_accuracy_against_mpmath():
    mpmath.mp.dps = 40
    rng = np.random.default_rng(8)
    xs = np.concatenate([rng.uniform(-1e-2, 1e-2, 2000), rng.uniform(-10, 10, 2000), [0.0, -0.0]])
    s, c = oracle.dsincos(xs)
    ws = max(ulp_err(v, mpmath.sin(mpmath.mpf(float(x)))) for x, v in zip(xs, s) if x != 0)
    wc = max(ulp_err(v, mpmath.cos(mpmath.mpf(float(x)))) for x, v in zip(xs, c))
    assert ws <= 2.0 and wc <= 2.0, (ws, wc)
    assert np.all(np.abs(s * s + c * c - 1.0) < 4e-16)


def test_shift_exact_grid_and_uniform():
    s = np.array([oracle.shift(9, step, 0) for step in range(4000)])
    assert np.all(s >= -0.5) and np.all(s < 0.5)
    q = s * 2.0 ** 24
    assert np.all(q == np.round(q))  # exact multiples of 2^-24: representable in FP32
    assert np.all(s.astype(np.float32).astype(np.float64) == s)
    for k in range(3):
        assert stats.kstest(s[:, k], "uniform", args=(-0.5, 1.0)).pvalue > 1e-3
    # the cell edge scales the shift
    assert np.all(oracle.shift(9, 3, 0, 2.0) == 2.0 * oracle.shift(9, 3, 0, 1.0))


def test_site_normals_are_standard_normal():
    z, flags = oracle.site_normals(11, 3, 0, 40000)
    assert flags == 0
    for k in range(3):
        assert stats.kstest(z[:, k], "norm").pvalue > 1e-3
    cov = np.cov(z.T)
    assert np.allclose(cov, np.eye(3), atol=0.03)
    # different replica -> different numbers
    z2, _ = oracle.site_normals(11, 3, 1, 10)
    assert not np.allclose(z[:10], z2)


def test_cell_axes_uniform_on_sphere():
    ax, flags = oracle.cell_axes(5, 2, 0, 40000)
    assert flags == 0
    assert np.allclose(np.linalg.norm(ax, axis=1), 1.0, atol=1e-15)
    # Archimedes: every Cartesian component of a uniform unit vector is U(-1,1)
    for k in range(3):
        assert stats.kstest(ax[:, k], "uniform", args=(-1.0, 2.0)).pvalue > 1e-3
    assert np.allclose(ax.T @ ax / len(ax), np.eye(3) / 3, atol=0.01)


def test_cell_axis_and_gamma_share_a_stream_independently():
    """A cell's axis and thermostat variate come from the same calls (the
    axis from call 0's halves 0 and 1, the variate's normal pair and test
    uniforms from halves 2-5 of each call): the axis is the same whether or
    not the variate is drawn, each is the one drawn alone, and the two are
    uncorrelated across cells."""
    n, k = 20000, 6.0
    ax, g, flags = oracle.cell_draws(23, 9, 1, k, n)
    assert flags == 0
    ax0, _ = oracle.cell_axes(23, 9, 1, n)
    g0, _ = oracle.gammas(23, 9, 1, k, n)
    assert np.array_equal(ax, ax0) and np.array_equal(g, g0)
    lim = 4.0 / math.sqrt(n)
    for comp in (ax[:, 0], ax[:, 1], ax[:, 2], ax[:, 2] ** 2):
        assert abs(stats.spearmanr(comp, g)[0]) < lim
    # drawn from 32-bit halves, both still follow their target distributions
    assert stats.kstest(g, "gamma", args=(k,)).pvalue > 1e-3
    assert stats.kstest(ax[:, 2], "uniform", args=(-1.0, 2.0)).pvalue > 1e-3


@pytest.mark.parametrize("k", [1.5, 6.0, 13.5, 30.0])
def test_gamma_sampler(k):
    g, flags = oracle.gammas(17, 4, 0, k, 30000)
    assert flags == 0
    assert stats.kstest(g, "gamma", args=(k,)).pvalue > 1e-3
    assert abs(g.mean() - k) < 4 * math.sqrt(k / len(g))
