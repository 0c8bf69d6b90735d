"""Pins for the oracle's level-crossing probability (Section 3.1, LCP after Poethkow et al.)."""

import mpmath
import numpy as np
import pytest
from scipy.stats import norm

import oracle as O


def _field(ny, nx, seed, sd=(0.05, 1.0)):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 1.0, (ny, nx)), rng.uniform(sd[0], sd[1], (ny, nx)) ** 2


def _marching_squares_crossed(d, c):
    """Textbook marching squares: 4-bit case index of corners >= c; the cell
    holds contour segments unless the case is 0 or 15."""
    b = (d >= c).astype(np.int64)
    case = b[:-1, :-1] | (b[:-1, 1:] << 1) | (b[1:, 1:] << 2) | (b[1:, :-1] << 3)
    return ((case != 0) & (case != 15)).astype(np.float64)


@pytest.mark.parametrize("c", [-0.3, 0.0, 0.4])
def test_zero_variance_is_marching_squares(c):
    mu, _ = _field(11, 14, seed=1)
    mu[3, 4] = c  # an exact tie: counts as above
    mu[7, 7] = c
    got = O.lcp(mu, np.zeros_like(mu), [c])[0]
    np.testing.assert_array_equal(got, _marching_squares_crossed(mu, c))


@pytest.mark.parametrize("z", [-3.0, -1.0, 0.0, 0.37, 2.5])
def test_iid_vertices_closed_form(z):
    m, s = 0.2, 0.7
    c = m - z * s
    mu = np.full((3, 4), m)
    var = np.full((3, 4), s * s)
    got = O.lcp(mu, var, [c])[0]
    p = norm.cdf(z)  # P(X >= c) for X ~ N(m, s^2) and c = m - z s
    want = 1.0 - p ** 4 - (1.0 - p) ** 4
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-15)


def test_all_corners_at_isovalue_gives_seven_eighths():
    got = O.lcp(np.full((2, 2), 1.5), np.full((2, 2), 0.04), [1.5])[0]
    assert got[0, 0] == 0.875


def test_range_symmetry_and_transpose():
    mu, var = _field(17, 23, seed=2)
    iso = [-1.0, -0.1, 0.0, 0.25, 2.0]
    L = O.lcp(mu, var, iso)
    assert np.all(L >= -1e-15) and np.all(L <= 1.0 + 1e-15)
    np.testing.assert_allclose(O.lcp(-mu, var, [-c for c in iso]), L, atol=1e-14)
    lt = O.lcp(mu.T, var.T, iso)
    np.testing.assert_allclose(lt, L.transpose(0, 2, 1), atol=1e-15)


def test_far_isovalue_vanishes():
    mu, var = _field(9, 9, seed=3)
    c = mu.max() + 12.0 * np.sqrt(var.max())
    assert np.all(O.lcp(mu, var, [c]) <= 1e-30)
    c = mu.min() - 12.0 * np.sqrt(var.max())
    assert np.all(O.lcp(mu, var, [c]) <= 1e-30)


def test_vertex_probs_mpmath_tails():
    """P(X >= c) and P(X < c) against 50-digit mpmath on the same float64
    inputs, deep into both tails.  Tolerance: the oracle rounds the erfc
    argument x = (c - mu)/(sqrt(var) sqrt 2) in about 5 float64 operations, and a
    relative error d in x moves erfc(x) by about 2 x^2 d relatively."""
    mpmath.mp.dps = 50
    rng = np.random.default_rng(4)
    mu = rng.normal(0, 1, 400)
    var = rng.uniform(0.01, 1.0, 400) ** 2
    z = rng.uniform(-12, 12, 400)
    c = mu + z * np.sqrt(var)
    for k in range(400):
        a, b = O.vertex_probs(mu[k], var[k], c[k])
        x = (mpmath.mpf(float(c[k])) - mpmath.mpf(float(mu[k]))) / (
            mpmath.sqrt(mpmath.mpf(float(var[k]))) * mpmath.sqrt(2))
        ea = mpmath.erfc(x) / 2
        eb = mpmath.erfc(-x) / 2
        rel = 1e-15 + 2.0 * (float(x) ** 2 + 1.0) * 5.0 * 2.0 ** -53
        assert abs(float(a) - float(ea)) <= rel * float(ea) + 1e-300
        assert abs(float(b) - float(eb)) <= rel * float(eb) + 1e-300


def test_lcp_against_mpmath_near_zero_and_one():
    """The FP64 literal 1 - A - B is within 1e-15 absolute of a 50-digit
    evaluation of the same definition, in the near-0 and near-1 bins."""
    mpmath.mp.dps = 50
    mu, var = _field(40, 40, seed=5, sd=(0.01, 0.3))
    iso = np.quantile(mu, [0.02, 0.5, 0.98])
    L = O.lcp(mu, var, iso)
    picks = []
    for k in range(len(iso)):
        for (j, i) in np.argwhere(L[k] < 1e-6)[:20]:
            picks.append((k, j, i))
        for (j, i) in np.argwhere(L[k] > 1 - 1e-6)[:20]:
            picks.append((k, j, i))
    assert len(picks) >= 20
    for k, j, i in picks:
        c = mpmath.mpf(float(iso[k]))
        A = mpmath.mpf(1); B = mpmath.mpf(1)
        for (jj, ii) in ((j, i), (j, i + 1), (j + 1, i), (j + 1, i + 1)):
            x = (c - mpmath.mpf(float(mu[jj, ii]))) / (mpmath.sqrt(mpmath.mpf(float(var[jj, ii]))) * mpmath.sqrt(2))
            A *= mpmath.erfc(x) / 2
            B *= mpmath.erfc(-x) / 2
        assert abs(float(L[k, j, i]) - float(1 - A - B)) <= 1e-15


def test_vertex_level_brute_force_all_cells():
    """Independent corner draws converge to the closed form on every cell."""
    mu, var = _field(6, 7, seed=6, sd=(0.2, 1.0))
    iso = [-0.2, 0.3]
    n = 40000
    L = O.lcp(mu, var, iso)
    E = O.mc_lcp_vertex(mu, var, iso, n, seed=7)
    se = np.sqrt(np.maximum(L * (1 - L), 1.0 / n) / n)
    z = np.abs(E - L) / se
    assert np.mean(z > 3.0) <= 0.01 + 1.0 / z.size
    chi2 = np.mean(z ** 2)
    assert chi2 < 1.0 + 5.0 * np.sqrt(2.0 / z.size)
