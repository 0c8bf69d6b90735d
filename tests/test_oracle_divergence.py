"""Pins for the oracle's Eq. 1-3 (Section 3.1) and the Fig. 2 worked example (Section 3.2)."""

import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig2_worked_example.txt")


def _fig2():
    nb, errs = {}, []
    for line in open(GOLD):
        line = line.split("#")[0].split()
        if not line:
            continue
        if line[0] == "mc_err":
            errs.append((int(line[1]), float(line[2]), float(line[3])))
        else:
            nb[line[0]] = (float(line[1]), float(line[2]))
    return nb, errs


def _fig2_grid():
    """3x3 grid whose centre vertex (1,1) has the Fig. 2 neighbours."""
    nb, _ = _fig2()
    mu_u = np.zeros((3, 3)); var_u = np.ones((3, 3))
    mu_v = np.zeros((3, 3)); var_v = np.ones((3, 3))
    mu_u[1, 0], var_u[1, 0] = nb["U_im1"][0], nb["U_im1"][1] ** 2
    mu_u[1, 2], var_u[1, 2] = nb["U_ip1"][0], nb["U_ip1"][1] ** 2
    mu_v[0, 1], var_v[0, 1] = nb["V_jm1"][0], nb["V_jm1"][1] ** 2
    mu_v[2, 1], var_v[2, 1] = nb["V_jp1"][0], nb["V_jp1"][1] ** 2
    return mu_u, var_u, mu_v, var_v


def test_fig2_worked_example_moments():
    # (6.40-5.98)/2 + (4.30-6.50)/2 = -0.89 and (0.96^2+0.38^2+0.94^2+0.65^2)/4 = 0.593025
    m, v = O.divergence_gaussian(*_fig2_grid(), 1.0, 1.0)
    assert m[1, 1] == pytest.approx(-0.89, abs=1e-14)
    assert v[1, 1] == pytest.approx(0.593025, abs=1e-14)


@pytest.mark.parametrize("n", [1000, 100000])
def test_fig2_monte_carlo_errors(n):
    """MC of the Eq. 1 stencil at the Fig. 2 neighbours lands within 3 standard
    errors of the analytic mean and standard deviation, and the paper's printed
    errors are of the size sampling noise allows at that count."""
    nb, errs = _fig2()
    rng = np.random.default_rng(20251001 + n)
    d = ((rng.normal(*nb["U_ip1"], n) - rng.normal(*nb["U_im1"], n)) / 2.0
         + (rng.normal(*nb["V_jp1"], n) - rng.normal(*nb["V_jm1"], n)) / 2.0)
    m, v = O.divergence_gaussian(*_fig2_grid(), 1.0, 1.0)
    mu, sd = m[1, 1], np.sqrt(v[1, 1])
    se_mean = sd / np.sqrt(n)
    se_sd = sd / np.sqrt(2.0 * (n - 1))
    assert abs(d.mean() - mu) < 3.0 * se_mean
    assert abs(d.std(ddof=1) - sd) < 3.0 * se_sd
    e_m, e_s = {k: (a, b) for k, a, b in errs}[n]
    assert e_m < 3.0 * se_mean and e_s < 3.0 * se_sd


def _rand_moments(ny, nx, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(0, 2, (ny, nx)), rng.uniform(0.01, 1.5, (ny, nx)),
            rng.normal(0, 2, (ny, nx)), rng.uniform(0.01, 1.5, (ny, nx)))


@pytest.mark.parametrize("shape", [(2, 2), (2, 5), (7, 2), (9, 13)])
def test_mean_equals_numpy_gradient(shape):
    mu_u, var_u, mu_v, var_v = _rand_moments(*shape, seed=sum(shape))
    dx, dy = 0.7, 1.9
    m, _ = O.divergence_gaussian(mu_u, var_u, mu_v, var_v, dx, dy)
    ref = (np.gradient(mu_u, dx, axis=1, edge_order=1)
           + np.gradient(mu_v, dy, axis=0, edge_order=1))
    np.testing.assert_allclose(m, ref, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(O.fd_divergence(mu_u, mu_v, dx, dy), ref, rtol=1e-13, atol=1e-13)


def test_linear_field_closed_form():
    ny, nx = 6, 9
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    dx, dy = 0.5, 2.0
    alpha, gamma = 1.7, -0.3
    u = alpha * x * dx + 3.0
    v = gamma * y * dy - 1.0
    m, _ = O.divergence_gaussian(u, np.zeros_like(u), v, np.zeros_like(v), dx, dy)
    np.testing.assert_allclose(m, alpha + gamma, atol=1e-13)


def test_uniform_sigma_closed_form():
    # dx = dy = h, sigma = s everywhere: s^2/h^2 inside, 2.5 s^2/h^2 on edges, 4 s^2/h^2 at corners
    ny, nx, s, h = 5, 6, 0.3, 0.25
    z = np.zeros((ny, nx))
    _, v = O.divergence_gaussian(z, np.full((ny, nx), s * s), z, np.full((ny, nx), s * s), h, h)
    k = s * s / (h * h)
    np.testing.assert_allclose(v[1:-1, 1:-1], k, rtol=1e-13)
    np.testing.assert_allclose(v[0, 1:-1], 2.5 * k, rtol=1e-13)
    np.testing.assert_allclose(v[-1, 1:-1], 2.5 * k, rtol=1e-13)
    np.testing.assert_allclose(v[1:-1, 0], 2.5 * k, rtol=1e-13)
    np.testing.assert_allclose(v[1:-1, -1], 2.5 * k, rtol=1e-13)
    for c in [(0, 0), (0, -1), (-1, 0), (-1, -1)]:
        assert v[c] == pytest.approx(4 * k, rel=1e-13)


def test_x_and_y_parts_are_separate():
    # only V varies along y: the x part must not see it, and vice versa
    ny, nx = 5, 7
    rng = np.random.default_rng(3)
    vv = rng.uniform(0.1, 1, (ny, nx))
    z = np.zeros((ny, nx))
    _, var_only_v = O.divergence_gaussian(z, z, z, vv, 1.0, 1.0)
    _, var_only_u = O.divergence_gaussian(z, vv, z, z, 1.0, 1.0)
    # row j=2 (interior): var from V uses rows 1 and 3 of the same column
    np.testing.assert_allclose(var_only_v[2], (vv[1] + vv[3]) / 4.0, rtol=1e-13)
    # column i=3 (interior): var from U uses columns 2 and 4 of the same row
    np.testing.assert_allclose(var_only_u[:, 3], (vv[:, 2] + vv[:, 4]) / 4.0, rtol=1e-13)


def test_transpose_invariance():
    mu_u, var_u, mu_v, var_v = _rand_moments(7, 10, seed=11)
    m, v = O.divergence_gaussian(mu_u, var_u, mu_v, var_v, 0.8, 1.3)
    mt, vt = O.divergence_gaussian(mu_v.T, var_v.T, mu_u.T, var_u.T, 1.3, 0.8)
    np.testing.assert_allclose(mt, m.T, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(vt, v.T, rtol=1e-13)


def test_spacing_scale():
    mu_u, var_u, mu_v, var_v = _rand_moments(6, 8, seed=12)
    m1, v1 = O.divergence_gaussian(mu_u, var_u, mu_v, var_v, 1.0, 1.0)
    a = 3.5
    m2, v2 = O.divergence_gaussian(mu_u, var_u, mu_v, var_v, a, a)
    np.testing.assert_allclose(m2, m1 / a, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(v2, v1 / a ** 2, rtol=1e-13)


def test_brute_force_sampling_every_vertex():
    """Draw the whole field many times, apply Eq. 1 per draw: the empirical mean
    and variance at every vertex (boundaries included) match Eq. 2 / Eq. 3 and
    their one-sided boundary forms within sampling error."""
    ny, nx, n = 4, 5, 200000
    mu_u, var_u, mu_v, var_v = _rand_moments(ny, nx, seed=13)
    dx, dy = 0.9, 1.2
    m, v = O.divergence_gaussian(mu_u, var_u, mu_v, var_v, dx, dy)
    rng = np.random.default_rng(14)
    acc = np.zeros((ny, nx)); acc2 = np.zeros((ny, nx))
    for _ in range(n // 5000):
        u = mu_u + np.sqrt(var_u) * rng.standard_normal((5000, ny, nx))
        w = mu_v + np.sqrt(var_v) * rng.standard_normal((5000, ny, nx))
        # Eq. 1 per draw via the library routine (first-order one-sided edges)
        d = (np.gradient(u, dx, axis=2, edge_order=1)
             + np.gradient(w, dy, axis=1, edge_order=1))
        acc += d.sum(0); acc2 += (d ** 2).sum(0)
    em = acc / n
    ev = acc2 / n - em ** 2
    assert np.all(np.abs(em - m) < 4.5 * np.sqrt(v / n))
    assert np.all(np.abs(ev / v - 1.0) < 4.5 * np.sqrt(2.0 / n) + 1e-3)


def test_f32_divergence_equals_f64_where_float32_is_exact():
    """Integer means and variances with power-of-two spacings make every
    float32 operation of Eq. 2-3 exact, so the float32 evaluation must equal
    the float64 definition (bit for bit for the mean; the variance up to the
    float64 definition's own rounding of sqrt(var) squared) -- a dropped term,
    a wrong neighbour or a wrong boundary coefficient cannot survive this."""
    rng = np.random.default_rng(21)
    for ny, nx, dx, dy in ((7, 9, 0.5, 2.0), (2, 2, 1.0, 1.0), (2, 13, 4.0, 0.25), (11, 2, 1.0, 0.5)):
        mu_u, mu_v = rng.integers(-1000, 1000, (2, ny, nx)).astype(np.float64)
        var_u, var_v = rng.integers(0, 1000, (2, ny, nx)).astype(np.float64)
        m64, v64 = O.divergence_gaussian(mu_u, var_u, mu_v, var_v, dx, dy)
        m32, v32 = O.divergence_gaussian_f32(mu_u, var_u, mu_v, var_v, dx, dy)
        assert m32.dtype == np.float32 and v32.dtype == np.float32
        np.testing.assert_array_equal(m32.astype(np.float64), m64)
        # the float64 definition squares sqrt(var) / h, which rounds twice
        np.testing.assert_allclose(v32.astype(np.float64), v64, rtol=4e-16, atol=0)


def test_f32_divergence_is_within_rounding_of_f64():
    rng = np.random.default_rng(22)
    ny, nx = 23, 31
    mu_u, mu_v = rng.normal(0, 1, (2, ny, nx))
    var_u, var_v = rng.uniform(0.01, 1, (2, ny, nx))
    m64, v64 = O.divergence_gaussian(mu_u, var_u, mu_v, var_v, 0.3, 1.7)
    m32, v32 = O.divergence_gaussian_f32(mu_u, var_u, mu_v, var_v, 0.3, 1.7)
    u = 2.0 ** -24
    scale = (np.abs(mu_u).max() / 0.3 + np.abs(mu_v).max() / 1.7) * 2
    assert np.max(np.abs(m32 - m64)) <= 8 * u * scale
    assert np.max(np.abs(v32 - v64) / v64) <= 8 * u
