"""Pins for the oracle's isocontour geometry (marching squares: the
mean-field contour and the spaghetti plot of Section 4)."""

import collections

import numpy as np
import pytest

import oracle as O


def _grid(ny, nx):
    return np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64))


def _cases(f, c):
    up = (f >= c)
    return (up[:-1, :-1] * 1 + up[:-1, 1:] * 2 + up[1:, 1:] * 4 + up[1:, :-1] * 8)


@pytest.mark.parametrize("a,b,d,c", [(0.3, 0.7, -1.0, 2.2), (-1.1, 0.2, 5.0, 1.3),
                                     (1.0, 0.0, 0.0, 3.5)])
def test_plane_gives_the_exact_line(a, b, d, c):
    x, y = _grid(9, 12)
    f = a * x + b * y + d
    s = O.marching_squares(f, c)
    assert len(s) == int(np.sum((_cases(f, c) != 0) & (_cases(f, c) != 15)))
    np.testing.assert_allclose(a * s[:, 0] + b * s[:, 1] + d, c, atol=1e-12)
    np.testing.assert_allclose(a * s[:, 2] + b * s[:, 3] + d, c, atol=1e-12)


def test_circle_is_a_closed_loop():
    x, y = _grid(30, 34)
    cx, cy, r = 16.3, 14.7, 9.2
    f = (x - cx) ** 2 + (y - cy) ** 2
    s = O.marching_squares(f, r * r)
    ends = collections.Counter()
    for x0, y0, x1, y1 in s:
        for p in ((x0, y0), (x1, y1)):
            # every point lies on a cell edge
            assert p[0] == round(p[0]) or p[1] == round(p[1])
            ends[(round(p[0], 9), round(p[1], 9))] += 1
    assert set(ends.values()) == {2}  # closed: every point joins two segments
    d = np.hypot(s[:, [0, 2]] - cx, s[:, [1, 3]] - cy)
    assert np.all(np.abs(d - r) < 0.02)  # linear interpolation of a quadratic


def test_crossed_cells_are_the_zero_variance_lcp():
    rng = np.random.default_rng(3)
    f = np.round(rng.normal(0, 1, (11, 13)), 1)  # ties at the isovalue occur
    for c in (0.0, 0.4, -1.2):
        cases = _cases(f, c)
        n_per_cell = np.where((cases == 0) | (cases == 15), 0,
                              np.where((cases == 5) | (cases == 10), 2, 1))
        assert len(O.marching_squares(f, c)) == n_per_cell.sum()
        ind = O.lcp(f, np.zeros_like(f), [c])[0]
        np.testing.assert_array_equal(n_per_cell > 0, ind == 1.0)


def test_row_counts_are_the_segments_of_each_row():
    """marching_squares_row_counts, from the case numbers alone, equals the
    number of segments marching_squares emits for each one-row band, on
    fields with ties at the isovalue and saddles, and its crossed cells are
    those of the zero-variance LCP."""
    rng = np.random.default_rng(5)
    fields = [np.round(rng.normal(0, 1, (9, 23)), 1),
              np.tile(np.array([[1.0, 0.0], [0.0, 1.0]]), (5, 6)),
              rng.normal(0, 1, (2, 40))]
    for f in fields:
        for c in (0.0, 0.3, 0.5, -1.1):
            n = O.marching_squares_row_counts(f, c)
            assert n.shape == (f.shape[0] - 1,)
            for j in range(f.shape[0] - 1):
                assert n[j] == len(O.marching_squares(f[j:j + 2], c))
            assert n.sum() == len(O.marching_squares(f, c))
            crossed = O.lcp(f, np.zeros_like(f), [c])[0] == 1.0
            assert np.all(n >= crossed.sum(axis=1)) and np.all(n <= 2 * crossed.sum(axis=1))


def test_saddles_follow_the_centre():
    f = np.array([[1.0, 0.0], [0.0, 1.0]])  # (0,0) and (1,1) above: case 5
    s = O.marching_squares(f, 0.5)  # centre 0.5 >= 0.5: the above corners join
    np.testing.assert_allclose(s, [[0.5, 0.0, 1.0, 0.5], [0.5, 1.0, 0.0, 0.5]])
    s = O.marching_squares(f, 0.6)  # centre below: the above corners are cut off
    np.testing.assert_allclose(s, [[0.0, 0.4, 0.4, 0.0], [1.0, 0.6, 0.6, 1.0]])
    g = np.array([[0.0, 1.0], [1.0, 0.0]])  # case 10
    s = O.marching_squares(g, 0.5)
    np.testing.assert_allclose(s, [[0.0, 0.5, 0.5, 0.0], [1.0, 0.5, 0.5, 1.0]])


def test_negating_field_and_isovalue_keeps_the_segments():
    rng = np.random.default_rng(8)
    f = rng.normal(0, 1, (14, 17))  # no exact ties
    key = lambda s: sorted(tuple(sorted([(round(a, 9), round(b, 9)), (round(c, 9), round(d, 9))]))
                           for a, b, c, d in s)
    for c in (0.1, -0.7):
        assert key(O.marching_squares(f, c)) == key(O.marching_squares(-f, -c))


def test_spaghetti_is_one_contour_per_member():
    rng = np.random.default_rng(2)
    U, V = rng.normal(0, 1, (3, 8, 9)), rng.normal(0, 1, (3, 8, 9))
    sp = O.spaghetti(U, V, 1.0, 1.0, 0.2)
    assert len(sp) == 3
    for u, v, s in zip(U, V, sp):
        np.testing.assert_array_equal(s, O.marching_squares(O.fd_divergence(u, v, 1.0, 1.0), 0.2))
