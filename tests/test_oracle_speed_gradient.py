"""Pins for the oracle's Red Sea pre-stage (Section 4): the members'
gradient-of-speed vectors and their Gaussian fit."""

import numpy as np
import pytest

import oracle as O


def _members(m, ny, nx, seed):
    rng = np.random.default_rng(seed)
    base_u = rng.normal(0, 1, (ny, nx))
    base_v = rng.normal(0, 1, (ny, nx))
    return (base_u + 0.3 * rng.normal(0, 1, (m, ny, nx)),
            base_v + 0.3 * rng.normal(0, 1, (m, ny, nx)))


@pytest.mark.parametrize("shape,h", [((7, 9), (1.0, 1.0)), ((2, 5), (0.5, 2.0)),
                                     ((6, 2), (3.0, 0.25))])
def test_is_numpy_gradient_of_hypot(shape, h):
    rng = np.random.default_rng(1)
    u, v = rng.normal(0, 1, shape), rng.normal(0, 1, shape)
    gx, gy = O.speed_gradient(u, v, *h)
    s = np.hypot(u, v)
    np.testing.assert_allclose(gx, np.gradient(s, h[0], axis=1, edge_order=1), rtol=1e-13,
                               atol=1e-13)
    np.testing.assert_allclose(gy, np.gradient(s, h[1], axis=0, edge_order=1), rtol=1e-13,
                               atol=1e-13)


def test_linear_speed_has_constant_gradient():
    """u = a x (a > 0, x >= 0), v = 0: the speed is a x, so every difference,
    central or one-sided, gives (a, 0)."""
    ny, nx, a = 5, 8, 0.7
    x = np.tile(np.arange(nx, dtype=np.float64), (ny, 1))
    gx, gy = O.speed_gradient(a * x * 0.5, 0 * x, 0.5, 1.0)
    np.testing.assert_allclose(gx, a, atol=1e-14)
    np.testing.assert_allclose(gy, 0.0, atol=1e-14)


def test_rotation_and_reflection_do_not_change_the_fit():
    U, V = _members(6, 8, 9, seed=2)
    ref = O.speed_gradient_moments(U, V, 1.0, 1.0, 1)
    th = 0.83
    rot = O.speed_gradient_moments(U * np.cos(th) - V * np.sin(th),
                                   U * np.sin(th) + V * np.cos(th), 1.0, 1.0, 1)
    ref_flip = O.speed_gradient_moments(-U, V, 1.0, 1.0, 1)
    for a, b, c in zip(ref, rot, ref_flip):
        np.testing.assert_allclose(b, a, rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(c, a, rtol=1e-13, atol=1e-14)


def test_identical_members_have_zero_spread():
    U, V = _members(1, 6, 7, seed=3)
    m = 4
    mg = O.speed_gradient_moments(np.repeat(U, m, 0), np.repeat(V, m, 0), 1.0, 2.0, 1)
    gx, gy = O.speed_gradient(U[0], V[0], 1.0, 2.0)
    np.testing.assert_allclose(mg[0], gx, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(mg[2], gy, rtol=1e-15, atol=1e-15)
    assert np.all(mg[1] < 1e-28) and np.all(mg[3] < 1e-28)


@pytest.mark.parametrize("ddof", [0, 1])
def test_fit_is_the_sample_mean_and_variance_of_the_gradients(ddof):
    U, V = _members(5, 4, 6, seed=4)
    g = [O.speed_gradient(u, v, 1.0, 1.0) for u, v in zip(U, V)]
    gx = np.stack([a for a, _ in g])
    gy = np.stack([b for _, b in g])
    mg = O.speed_gradient_moments(U, V, 1.0, 1.0, ddof)
    np.testing.assert_allclose(mg[0], gx.mean(0), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(mg[1], gx.var(0, ddof=ddof), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(mg[2], gy.mean(0), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(mg[3], gy.var(0, ddof=ddof), rtol=1e-12, atol=1e-14)
