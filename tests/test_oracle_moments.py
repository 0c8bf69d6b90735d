"""Pins for the oracle's per-point Gaussian fit over ensemble members (Sections 3 and 4)."""

import numpy as np
import pytest

import oracle as O
import synth


@pytest.mark.parametrize("ddof", [0, 1])
def test_matches_numpy_mean_var(ddof):
    rng = np.random.default_rng(1)
    u = rng.normal(3.0, 2.0, (15, 9, 11))
    v = rng.normal(-1.0, 0.5, (15, 9, 11))
    mu, vu, mv, vv = O.moments(u, v, ddof)
    np.testing.assert_allclose(mu, u.mean(0), rtol=1e-14)
    np.testing.assert_allclose(vu, u.var(0, ddof=ddof), rtol=1e-12)
    np.testing.assert_allclose(mv, v.mean(0), rtol=1e-14)
    np.testing.assert_allclose(vv, v.var(0, ddof=ddof), rtol=1e-12)


def test_constant_members_have_zero_variance():
    u = np.full((20, 4, 5), 7.25)
    mu, vu, _, vv = O.moments(u, -u, 1)
    assert np.all(mu == 7.25) and np.all(vu == 0.0) and np.all(vv == 0.0)


def test_shift_invariance():
    rng = np.random.default_rng(2)
    u = rng.normal(0, 1, (8, 3, 3))
    a = O.moments(u, u, 1)
    b = O.moments(u + 100.0, u - 100.0, 1)
    np.testing.assert_allclose(b[0], a[0] + 100.0, rtol=1e-13)
    np.testing.assert_allclose(b[2], a[2] - 100.0, rtol=1e-13)
    np.testing.assert_allclose(b[1], a[1], rtol=1e-9)


def test_needs_more_members_than_ddof():
    with pytest.raises(ValueError):
        O.moments(np.zeros((1, 2, 2)), np.zeros((1, 2, 2)), 1)


def test_recovers_generator_truth():
    """Fitted moments of a synthetic ensemble match the generator's base field
    and spread maps within sampling error (sd/sqrt(M), sqrt(2/(M-1)))."""
    e = synth.gen_ensemble(40, 60, 50, seed=3, n_features=4)
    mu, vu, mv, vv = O.moments(e["u_members"], e["v_members"], 1)
    m = 50
    zu = (mu - e["u_base"]) / (e["std_u"] / np.sqrt(m))
    zv = (mv - e["v_base"]) / (e["std_v"] / np.sqrt(m))
    assert np.mean(np.abs(zu) > 3) < 0.01 and np.mean(np.abs(zv) > 3) < 0.01
    ru = vu / e["std_u"] ** 2 - 1.0
    assert np.mean(np.abs(ru) > 3 * np.sqrt(2.0 / (m - 1))) < 0.01
