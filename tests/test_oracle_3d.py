"""Pins for the oracle's 3D extension (the paper's future work, Section 5):
the divergence Gaussian with a z term and the 8-corner level-crossing
probability.  Each check ties the oracle to something other than itself:
numpy.gradient, closed forms, the pinned 2D oracle, brute-force sampling."""

import itertools

import numpy as np
import pytest
from scipy.stats import norm

import oracle as O
import synth


def _field(nz, ny, nx, seed=3, sigma=(0.05, 0.5)):
    f = synth.gen_moments_3d(nz, ny, nx, seed, sigma=sigma)
    return [f[k] for k in ("mean_u", "var_u", "mean_v", "var_v", "mean_w", "var_w")]


@pytest.mark.parametrize("shape,h", [((7, 9, 11), (1.0, 1.0, 1.0)), ((2, 5, 3), (0.5, 2.0, 1.5)),
                                     ((4, 2, 2), (1.0, 0.25, 3.0))])
def test_mean_is_numpy_gradient(shape, h):
    mu_u, var_u, mu_v, var_v, mu_w, var_w = _field(*shape)
    dx, dy, dz = h
    m, _ = O.divergence_gaussian_3d(mu_u, var_u, mu_v, var_v, mu_w, var_w, dx, dy, dz)
    ref = (np.gradient(mu_u, dx, axis=2, edge_order=1) + np.gradient(mu_v, dy, axis=1, edge_order=1)
           + np.gradient(mu_w, dz, axis=0, edge_order=1))
    np.testing.assert_allclose(m, ref, rtol=1e-13, atol=1e-13)


def test_uniform_spread_closed_forms():
    """sigma = s at every point and component, step h on every axis: each axis
    adds s^2/(2h^2) at an interior index and 2 s^2/h^2 at a boundary index,
    so a vertex with b boundary axes has variance (3 + 3b) s^2 / (2 h^2)."""
    nz, ny, nx, s, h = 5, 6, 7, 0.3, 0.5
    one = np.ones((nz, ny, nx))
    _, v = O.divergence_gaussian_3d(0 * one, s * s * one, 0 * one, s * s * one, 0 * one,
                                    s * s * one, h, h, h)
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        b = (k in (0, nz - 1)) + (j in (0, ny - 1)) + (i in (0, nx - 1))
        assert v[k, j, i] == pytest.approx((3 + 3 * b) * s * s / (2 * h * h), rel=1e-14)


def test_linear_field_has_constant_divergence():
    nz, ny, nx = 4, 5, 6
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    al, ga, ep = 0.7, -1.3, 0.4
    zero = np.zeros((nz, ny, nx))
    m, _ = O.divergence_gaussian_3d(al * x * 0.5, zero, ga * y * 2.0, zero, ep * z * 1.5, zero,
                                    0.5, 2.0, 1.5)
    np.testing.assert_allclose(m, al + ga + ep, atol=1e-13)


def test_reduces_to_the_2d_oracle():
    """U and V constant along z and W deterministic zero: every z-slice holds
    the 2D divergence Gaussian of Eq. 2 and Eq. 3."""
    f = synth.gen_moments(9, 13, seed=8)
    nz = 3
    rep = [np.repeat(f[k][None], nz, axis=0) for k in ("mean_u", "var_u", "mean_v", "var_v")]
    zero = np.zeros_like(rep[0])
    m3, v3 = O.divergence_gaussian_3d(*rep, zero, zero, 1.0, 0.5, 2.0)
    m2, v2 = O.divergence_gaussian(f["mean_u"], f["var_u"], f["mean_v"], f["var_v"], 1.0, 0.5)
    for k in range(nz):
        np.testing.assert_allclose(m3[k], m2, rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(v3[k], v2, rtol=1e-15, atol=1e-15)


def test_swapping_x_and_z_transposes():
    mu_u, var_u, mu_v, var_v, mu_w, var_w = _field(4, 5, 6)
    m, v = O.divergence_gaussian_3d(mu_u, var_u, mu_v, var_v, mu_w, var_w, 0.5, 1.0, 2.0)
    t = lambda a: np.ascontiguousarray(a.transpose(2, 1, 0))
    mt, vt = O.divergence_gaussian_3d(t(mu_w), t(var_w), t(mu_v), t(var_v), t(mu_u), t(var_u),
                                      2.0, 1.0, 0.5)
    np.testing.assert_allclose(mt, t(m), rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(vt, t(v), rtol=1e-14, atol=1e-14)
    iso = [-0.3, 0.1]
    L = O.lcp_3d(m, v, iso)
    Lt = O.lcp_3d(mt, vt, iso)
    np.testing.assert_allclose(Lt, L.transpose(0, 3, 2, 1), rtol=1e-13, atol=1e-15)


def test_iid_corners_closed_form():
    """All vertices N(m, s^2): LCP = 1 - Phi(z)^8 - (1 - Phi(z))^8 with
    z = (m - c)/s; at c = m exactly 1 - 2/256."""
    m, s = 0.3, 0.7
    mu = np.full((3, 4, 5), m)
    var = np.full((3, 4, 5), s * s)
    cs = [m, m - 0.4, m + 1.1, m - 2.5]
    L = O.lcp_3d(mu, var, cs)
    for q, c in enumerate(cs):
        p = norm.cdf((m - c) / s)
        np.testing.assert_allclose(L[q], 1 - p ** 8 - (1 - p) ** 8, rtol=1e-12, atol=1e-15)
    assert np.all(L[0] == 1.0 - 2.0 / 256.0)


def test_zero_variance_is_marching_cubes():
    """Deterministic corners: the LCP is the crossing indicator of the mean
    field, counted here corner by corner (>= is above)."""
    rng = np.random.default_rng(4)
    mu = np.round(rng.normal(0, 1, (5, 6, 7)), 1)  # ties at the isovalues occur
    var = np.zeros_like(mu)
    for c in (0.0, 0.3, -0.7):
        L = O.lcp_3d(mu, var, [c])[0]
        for k, j, i in itertools.product(range(4), range(5), range(6)):
            up = [mu[k + a, j + b, i + d] >= c for a in (0, 1) for b in (0, 1) for d in (0, 1)]
            assert L[k, j, i] == (0.0 if all(up) or not any(up) else 1.0)


def test_range_symmetry_and_far_isovalues():
    mu_u, var_u, mu_v, var_v, mu_w, var_w = _field(6, 7, 8)
    m, v = O.divergence_gaussian_3d(mu_u, var_u, mu_v, var_v, mu_w, var_w, 1.0, 1.0, 1.0)
    iso = np.array([-0.5, 0.0, 0.4])
    L = O.lcp_3d(m, v, iso)
    assert np.all((L >= 0) & (L <= 1))
    np.testing.assert_allclose(O.lcp_3d(-m, v, -iso), L, rtol=1e-12, atol=1e-15)
    far = m.max() + 12 * np.sqrt(v.max())
    assert O.lcp_3d(m, v, [far, -far + 2 * m.min()]).max() <= 1e-30


def test_vertex_brute_force_converges_everywhere():
    mu_u, var_u, mu_v, var_v, mu_w, var_w = _field(4, 5, 6, seed=9)
    m, v = O.divergence_gaussian_3d(mu_u, var_u, mu_v, var_v, mu_w, var_w, 1.0, 1.0, 1.0)
    iso = [float(np.median(m)), float(np.quantile(m, 0.8))]
    S = 4000
    L = O.lcp_3d(m, v, iso)
    E = O.mc_lcp_3d_vertex(m, v, iso, S, seed=5)
    se = np.sqrt(np.maximum(L * (1 - L), 1.0 / S) / S)
    z = np.abs(E - L) / se
    assert np.mean(z > 3.0 + 1.0 / (S * se)) <= 0.01
    assert np.mean(z ** 2) < 1.5


def test_vector_monte_carlo_converges_on_interior_cells():
    """Interior hexahedra (1 <= i <= nx-3, likewise j, k) difference disjoint
    samples at their 8 corners, so sampling the vectors estimates exactly the
    independent-corner LCP there."""
    nz, ny, nx = 6, 6, 7
    f = _field(nz, ny, nx, seed=12, sigma=(0.1, 0.5))
    m, v = O.divergence_gaussian_3d(*f, 1.0, 1.0, 1.0)
    iso = [float(np.median(m))]
    S = 3000
    L = O.lcp_3d(m, v, iso)
    E = O.mc_lcp_3d(*f, 1.0, 1.0, 1.0, iso, S, seed=21)
    inner = np.zeros(L.shape[1:], bool)
    inner[1:nz - 2, 1:ny - 2, 1:nx - 2] = True
    se = np.sqrt(np.maximum(L * (1 - L), 1.0 / S) / S)
    z = (np.abs(E - L) / se)[:, inner]
    assert np.sum(z > 3.0 + 1.0 / (S * se[:, inner])) <= max(1, int(0.01 * z.size))
    assert np.mean(z ** 2) < 1.5


def test_f32_divergence_3d_equals_f64_where_float32_is_exact():
    rng = np.random.default_rng(31)
    for shape, h in (((5, 6, 7), (0.5, 2.0, 1.0)), ((2, 2, 2), (1.0, 1.0, 1.0)),
                     ((3, 2, 9), (4.0, 0.25, 0.5))):
        planes = []
        for _ in range(3):
            planes += [rng.integers(-1000, 1000, shape).astype(np.float64),
                       rng.integers(0, 1000, shape).astype(np.float64)]
        m64, v64 = O.divergence_gaussian_3d(*planes, *h)
        m32, v32 = O.divergence_gaussian_3d_f32(*planes, *h)
        assert m32.dtype == np.float32
        np.testing.assert_array_equal(m32.astype(np.float64), m64)
        # the float64 definition squares sqrt(var) / h, which rounds twice
        np.testing.assert_allclose(v32.astype(np.float64), v64, rtol=4e-16, atol=0)


def test_f32_divergence_3d_is_within_rounding_of_f64():
    rng = np.random.default_rng(32)
    shape = (6, 7, 8)
    planes = []
    for _ in range(3):
        planes += [rng.normal(0, 1, shape), rng.uniform(0.01, 1, shape)]
    m64, v64 = O.divergence_gaussian_3d(*planes, 0.7, 1.1, 1.9)
    m32, v32 = O.divergence_gaussian_3d_f32(*planes, 0.7, 1.1, 1.9)
    u = 2.0 ** -24
    assert np.max(np.abs(m32 - m64)) <= 12 * u * 3 * (1 / 0.7 + 1 / 1.1 + 1 / 1.9) * 4
    assert np.max(np.abs(v32 - v64) / v64) <= 12 * u
