"""Plain FP64 oracle of the probabilistic local-divergence path.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

Grid convention (the reading of Section 3.1 used throughout): i is the x index
(0 <= i < nx), j the y index (0 <= j < ny); arrays are row-major [ny][nx] with
x fastest.  U is the x component and V the y component of the uncertain vector
field F = (U, V); U_{i+-1} means U at (i+-1, j) and V_{j+-1} means V at
(i, j+-1).  Cell (i, j) has corners (i,j), (i+1,j), (i,j+1), (i+1,j+1).

Parity status per function:
  moments            pinned (numpy mean/var, closed forms, invariants)
  fd_divergence      pinned (numpy.gradient, linear fields)
  speed_gradient     pinned (numpy.hypot + numpy.gradient, linear speed,
                     rotation and reflection invariance)
  speed_gradient_moments  pinned through speed_gradient and moments, plus
                     identical members (zero variance)
  divergence_gaussian pinned (Fig. 2 worked example, numpy.gradient, closed forms,
                      brute-force sampling)
  divergence_gaussian_f32  pinned to divergence_gaussian: equal on inputs where
                      every float32 operation is exact, within float32
                      rounding elsewhere
  lcp                pinned (marching-squares limit, i.i.d. closed form, symmetry,
                      brute-force sampling, mpmath tails)
  philox4x32_10      pinned (published known-answer vectors, rocRAND routine)
  box_muller         pinned (closed form at chosen inputs, normality tests)
  marching_squares   pinned (planes: every point on the exact line; circles:
                     closed loops, every point shared by two segments; crossed
                     cells = the zero-variance LCP indicator; saddles)
  spaghetti          marching_squares of fd_divergence per member
  mc_lcp             vector mode: pinned statistically against lcp on interior
                     cells; vertex mode: against lcp on every cell, and exactly
                     against the marching-squares indicator at zero variance.
                     A single MC draw has no closed form to pin to.
"""

from __future__ import annotations

import numpy as np
from scipy.special import erfc

# ---------------------------------------------------------------------------
# (a) Gaussian fit per point (Section 3: each component independently
#     N(mu, sigma^2); Section 4 fits it over 15 or 20 ensemble members).
#     The paper does not name the estimator; the reading is the sample mean
#     and the sample variance with ddof in {0, 1} (default 1, unbiased).
# ---------------------------------------------------------------------------

def moments(u_members, v_members, ddof: int = 1):
    """Two-pass FP64 mean and variance over the member axis (axis 0).

    mu = (1/M) sum_m x_m;  sigma^2 = sum_m (x_m - mu)^2 / (M - ddof).
    Returns (mean_u, var_u, mean_v, var_v), each [ny][nx] float64."""
    out = []
    for x in (u_members, v_members):
        x = np.asarray(x, dtype=np.float64)
        m = x.shape[0]
        if m <= ddof:
            raise ValueError("need more members than ddof")
        mu = x.sum(axis=0) / m
        var = ((x - mu[None]) ** 2).sum(axis=0) / (m - ddof)
        out += [mu, var]
    return tuple(out)


# ---------------------------------------------------------------------------
# (b) Finite-difference divergence, Eq. 1: central differences inside,
#     forward / backward differences at the boundary (Section 3.1).
#     The order of the one-sided differences is not stated; the reading is
#     first order: (f_1 - f_0)/h at the low edge, (f_{n-1} - f_{n-2})/h at the
#     high edge.
# ---------------------------------------------------------------------------

def _ddx(f, h):
    """Derivative along x (axis 1) by Eq. 1's differences, float64."""
    f = np.asarray(f, np.float64)
    nx = f.shape[1]
    d = np.empty_like(f)
    d[:, 1:nx - 1] = (f[:, 2:] - f[:, :nx - 2]) / (2.0 * h)
    d[:, 0] = (f[:, 1] - f[:, 0]) / h
    d[:, nx - 1] = (f[:, nx - 1] - f[:, nx - 2]) / h
    return d


def fd_divergence(u, v, dx: float, dy: float):
    """Eq. 1 applied to one deterministic field (u, v): du/dx + dv/dy."""
    return _ddx(u, dx) + _ddx(np.asarray(v, np.float64).T, dy).T


def divergence_gaussian(mean_u, var_u, mean_v, var_v, dx: float, dy: float):
    """Eq. 2 (mean) and Eq. 3 (variance) of the divergence at every vertex.

    Inside, Eq. 2 and Eq. 3 as printed:
      mu  = mu^U_{i+1}/(2dx) - mu^U_{i-1}/(2dx) + mu^V_{j+1}/(2dy) - mu^V_{j-1}/(2dy)
      var = (s^U_{i+1}/(2dx))^2 + (s^U_{i-1}/(2dx))^2 + (s^V_{j+1}/(2dy))^2 + (s^V_{j-1}/(2dy))^2
    At a boundary the difference of Eq. 1 is one-sided with step h instead of
    2h; the same independence argument then gives, e.g. at i = 0,
      mu_x = (mu^U_1 - mu^U_0)/dx,  var_x = (s^U_1)^2/dx^2 + (s^U_0)^2/dx^2.
    Returns (div_mean, div_var), each [ny][nx] float64."""
    mu_u = np.asarray(mean_u, np.float64)
    mu_v = np.asarray(mean_v, np.float64)
    s_u = np.sqrt(np.asarray(var_u, np.float64))
    s_v = np.sqrt(np.asarray(var_v, np.float64))
    ny, nx = mu_u.shape

    mean = np.zeros((ny, nx), np.float64)
    var = np.zeros((ny, nx), np.float64)
    # x part, column by column over i
    for i in range(nx):
        if 0 < i < nx - 1:
            lo, hi, h = i - 1, i + 1, 2.0 * dx
        elif i == 0:
            lo, hi, h = 0, 1, dx
        else:
            lo, hi, h = nx - 2, nx - 1, dx
        mean[:, i] += mu_u[:, hi] / h - mu_u[:, lo] / h
        var[:, i] += (s_u[:, hi] / h) ** 2 + (s_u[:, lo] / h) ** 2
    # y part, row by row over j
    for j in range(ny):
        if 0 < j < ny - 1:
            lo, hi, h = j - 1, j + 1, 2.0 * dy
        elif j == 0:
            lo, hi, h = 0, 1, dy
        else:
            lo, hi, h = ny - 2, ny - 1, dy
        mean[j, :] += mu_v[hi, :] / h - mu_v[lo, :] / h
        var[j, :] += (s_v[hi, :] / h) ** 2 + (s_v[lo, :] / h) ** 2
    return mean, var


# ---------------------------------------------------------------------------
# (b') The Red Sea pre-stage (Section 4): for each ensemble member, the
#      pixelwise gradient of the velocity magnitude; the gradient vectors are
#      the field whose divergence uncertainty is analysed (sources of the
#      gradient of speed mark vortex cores).  The paper does not give the
#      difference scheme; the reading is Eq. 1's (central inside, first-order
#      one-sided at the boundary), and the Gaussian fit is moments() applied
#      to the members' gradient vectors.
# ---------------------------------------------------------------------------

def speed_gradient(u, v, dx: float, dy: float):
    """Gradient (gx, gy) of the speed sqrt(u^2 + v^2) of one member, [ny][nx]
    float64 each, by Eq. 1's differences."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    s = np.sqrt(u * u + v * v)
    return _ddx(s, dx), _ddx(s.T, dy).T


def speed_gradient_moments(u_members, v_members, dx: float, dy: float, ddof: int = 1):
    """Per-point Gaussian fit of the members' speed-gradient vectors:
    (mean_gx, var_gx, mean_gy, var_gy), [ny][nx] float64 each."""
    gx, gy = [], []
    for u, v in zip(u_members, v_members):
        a, b = speed_gradient(u, v, dx, dy)
        gx.append(a)
        gy.append(b)
    return moments(np.stack(gx), np.stack(gy), ddof)


# ---------------------------------------------------------------------------
# (c) Level-crossing probability (Section 3.1, after Poethkow et al.): the
#     probability that the c-isocontour crosses a cell whose four corners hold
#     independent Gaussians N(mu_k, sigma_k^2).  The contour crosses unless all
#     four corners lie on the same side of c, so
#         LCP = 1 - prod_k P(X_k >= c) - prod_k P(X_k < c).
#     Ties follow the marching-squares convention: a corner is "above" iff its
#     value >= c.  With sigma_k = 0 the corner is deterministic.
# ---------------------------------------------------------------------------

def vertex_probs(mu, var, c: float):
    """(a, b) = (P(X >= c), P(X < c)) for X ~ N(mu, var), elementwise float64."""
    mu = np.asarray(mu, np.float64)
    var = np.asarray(var, np.float64)
    sd = np.sqrt(var)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = 0.5 * erfc((c - mu) / (sd * np.sqrt(2.0)))
        b = 0.5 * erfc((mu - c) / (sd * np.sqrt(2.0)))
    det = sd == 0.0
    a = np.where(det, np.where(mu >= c, 1.0, 0.0), a)
    b = np.where(det, np.where(mu >= c, 0.0, 1.0), b)
    bad = np.isnan(mu) | np.isnan(var)
    a = np.where(bad, np.nan, a)
    b = np.where(bad, np.nan, b)
    return a, b


def lcp(div_mean, div_var, isovalues):
    """Closed-form LCP maps [K][ny-1][nx-1] float64 from the vertex Gaussians."""
    mu = np.asarray(div_mean, np.float64)
    var = np.asarray(div_var, np.float64)
    ny, nx = mu.shape
    iso = np.atleast_1d(np.asarray(isovalues, np.float64))
    out = np.empty((iso.size, ny - 1, nx - 1), np.float64)
    for k, c in enumerate(iso):
        a, b = vertex_probs(mu, var, c)
        corners_a = (a[:-1, :-1], a[:-1, 1:], a[1:, :-1], a[1:, 1:])
        corners_b = (b[:-1, :-1], b[:-1, 1:], b[1:, :-1], b[1:, 1:])
        all_above = corners_a[0] * corners_a[1] * corners_a[2] * corners_a[3]
        all_below = corners_b[0] * corners_b[1] * corners_b[2] * corners_b[3]
        out[k] = 1.0 - all_above - all_below
    return out


# ---------------------------------------------------------------------------
# (d) Monte Carlo LCP, the paper's comparison (Section 3.2 and Section 4):
#     draw samples of the uncertain vectors at every grid point, form the
#     divergence of each sample by Eq. 1, count per cell how often the
#     c-isocontour crosses it, divide by the sample count.
#
#     The paper names no random number generator.  Reading: Philox4x32-10
#     (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,
#     3", SC 2011) keyed by the 64-bit seed, with counter
#     (point index p = j*nx + i, sample pair q = s // 2, 0, 0); its four output
#     words feed two Box-Muller transforms (Box & Muller 1958): words (w0, w1)
#     give (U, V) standard normals of sample 2q, words (w2, w3) of sample 2q+1.
# ---------------------------------------------------------------------------

_PHILOX_M0 = np.uint64(0xD2511F53)
_PHILOX_M1 = np.uint64(0xCD9E8D57)
_PHILOX_W0 = 0x9E3779B9
_PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Philox4x32 with 10 rounds on uint32 arrays (c0..c3) and a 2-word key.

    One round: (hi0, lo0) = M0 * x0 and (hi1, lo1) = M1 * x2 as 64-bit products;
    new state = (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0).  Between rounds the key
    advances by the Weyl constants (W0, W1) modulo 2^32."""
    x0 = np.asarray(c0, np.uint32).astype(np.uint64)
    x1 = np.asarray(c1, np.uint32).astype(np.uint64)
    x2 = np.asarray(c2, np.uint32).astype(np.uint64)
    x3 = np.asarray(c3, np.uint32).astype(np.uint64)
    ka, kb = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r > 0:
            ka = (ka + _PHILOX_W0) & 0xFFFFFFFF
            kb = (kb + _PHILOX_W1) & 0xFFFFFFFF
        p0 = _PHILOX_M0 * x0
        p1 = _PHILOX_M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(ka), lo1, hi0 ^ x3 ^ np.uint64(kb), lo0)
    return tuple(w.astype(np.uint32) for w in (x0, x1, x2, x3))


def box_muller(wa, wb):
    """Two standard normals from two uint32 words, float64.

    u1 = (wa + 1) / 2^32 in (0, 1], u2 = wb / 2^32 in [0, 1);
    r = sqrt(-2 ln u1), z0 = r cos(2 pi u2), z1 = r sin(2 pi u2)."""
    u1 = (np.asarray(wa, np.float64) + 1.0) / 4294967296.0
    u2 = np.asarray(wb, np.float64) / 4294967296.0
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)


def _normals(n_points: int, s: int, seed: int, first: int = 0):
    """Standard normals (zu, zv) of sample s at points first .. first+n_points-1."""
    p = (np.arange(n_points, dtype=np.uint64) + np.uint64(first)).astype(np.uint32)
    q = np.full(n_points, s // 2, np.uint32)
    zero = np.zeros(n_points, np.uint32)
    w0, w1, w2, w3 = philox4x32_10(p, q, zero, zero, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return box_muller(w0, w1) if s % 2 == 0 else box_muller(w2, w3)


def mc_sample_field(mean_u, var_u, mean_v, var_v, s: int, seed: int, first_point: int = 0):
    """Sample s of the uncertain field: U = mu_u + sigma_u zu, V = mu_v + sigma_v zv (float64).
    first_point: the index of the planes' first point in a larger grid (the
    rows of a band of that grid), so that each point draws its own samples."""
    mu_u = np.asarray(mean_u, np.float64)
    ny, nx = mu_u.shape
    zu, zv = _normals(ny * nx, s, seed, first_point)
    u = mu_u + np.sqrt(np.asarray(var_u, np.float64)) * zu.reshape(ny, nx)
    v = np.asarray(mean_v, np.float64) + np.sqrt(np.asarray(var_v, np.float64)) * zv.reshape(ny, nx)
    return u, v


def _vertex_normals(n_points: int, s: int, seed: int):
    """Standard normal of sample s at vertices 0..n_points-1 for vertex-level
    sampling: counter (vertex index p, s // 4, 1, 0) -- the third word 1 keeps
    these streams apart from the vector-level ones -- with Box-Muller on
    (w0, w1) giving samples 4q and 4q+1 and on (w2, w3) samples 4q+2, 4q+3."""
    p = np.arange(n_points, dtype=np.uint64).astype(np.uint32)
    q = np.full(n_points, s // 4, np.uint32)
    one = np.ones(n_points, np.uint32)
    zero = np.zeros(n_points, np.uint32)
    w0, w1, w2, w3 = philox4x32_10(p, q, one, zero, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    pair = box_muller(w0, w1) if (s % 4) < 2 else box_muller(w2, w3)
    return pair[s % 2]


def divergence_gaussian_f32(mean_u, var_u, mean_v, var_v, dx: float, dy: float):
    """Eq. 2 and Eq. 3 with every operation rounded to float32, in the order
    mean = (mu_r - mu_l) cm_x + (mv_r - mv_l) cm_y and
    var = (var_r + var_l) cv_x + (var_r + var_l) cv_y, where cm = 1/(2h)
    inside and 1/h on the boundary and cv = 1/(4h^2) or 1/h^2, each rounded
    once from float64.  Returns float32 planes: the divergence Gaussians a
    float32 implementation that rounds in this order holds, bit for bit --
    the input for checking its later steps (the crossing decisions of the
    Monte Carlo, the relative accuracy of tiny LCP values) in its own
    precision."""
    f = np.float32
    mu_u, s2_u = np.asarray(mean_u, f), np.asarray(var_u, f)
    mu_v, s2_v = np.asarray(mean_v, f), np.asarray(var_v, f)
    ny, nx = mu_u.shape
    i, j = np.arange(nx), np.arange(ny)
    xl, xr = np.maximum(i - 1, 0), np.minimum(i + 1, nx - 1)
    yl, yr = np.maximum(j - 1, 0), np.minimum(j + 1, ny - 1)
    bx, by = (i == 0) | (i == nx - 1), (j == 0) | (j == ny - 1)
    cxm = np.where(bx, f(1.0 / dx), f(1.0 / (2.0 * dx))).astype(f)[None, :]
    cxv = np.where(bx, f(1.0 / (dx * dx)), f(1.0 / (4.0 * dx * dx))).astype(f)[None, :]
    cym = np.where(by, f(1.0 / dy), f(1.0 / (2.0 * dy))).astype(f)[:, None]
    cyv = np.where(by, f(1.0 / (dy * dy)), f(1.0 / (4.0 * dy * dy))).astype(f)[:, None]
    mx = (mu_u[:, xr] - mu_u[:, xl]) * cxm
    my = (mu_v[yr, :] - mu_v[yl, :]) * cym
    vx = (s2_u[:, xr] + s2_u[:, xl]) * cxv
    vy = (s2_v[yr, :] + s2_v[yl, :]) * cyv
    mean = mx + my
    var = vx + vy
    return mean, var


def _crossed(d, c):
    """Cells whose four corners are not all on one side of c (>= is above)."""
    up = d >= c
    a = up[:-1, :-1].astype(np.int8) + up[:-1, 1:] + up[1:, :-1] + up[1:, 1:]
    return (a != 0) & (a != 4)


def mc_lcp(mean_u, var_u, mean_v, var_v, dx: float, dy: float, isovalues,
           n_samples: int, seed: int, precision: str = "f64", mode: str = "vector",
           first_point: int = 0):
    """MC LCP maps [K][ny-1][nx-1] (crossing counts / n_samples).

    mode="vector" (the paper's sampling, Sections 3.2 and 4): each sample
    draws U and V at every grid point and takes the divergence by Eq. 1.
    mode="vertex": each sample draws every vertex divergence on its own from
    N(mu, var) of Eq. 2-3, so the four corners of a cell are independent even
    where the one-sided boundary differences share grid points -- the closed
    form's model, to which this mode converges on every cell.

    precision="f64": every step in float64 (the definition).
    precision="f32": the same steps with the sample field, the divergence and
    the crossing test rounded to float32 -- the precision in which a float32
    implementation takes the crossing decision.  The normals themselves are
    computed in float64 and rounded once.

    first_point (vector mode): the index of the planes' first point in a
    larger grid whose samples these are (see mc_lcp_rows)."""
    iso = np.atleast_1d(np.asarray(isovalues, np.float64))
    mu_u = np.asarray(mean_u, np.float64)
    ny, nx = mu_u.shape
    counts = np.zeros((iso.size, ny - 1, nx - 1), np.int64)
    if mode == "vertex":
        if precision == "f64":
            m, v = divergence_gaussian(mean_u, var_u, mean_v, var_v, dx, dy)
            sd = np.sqrt(v)
            for s in range(n_samples):
                d = m + sd * _vertex_normals(ny * nx, s, seed).reshape(ny, nx)
                for k, c in enumerate(iso):
                    counts[k] += _crossed(d, c)
        elif precision == "f32":
            f = np.float32
            m, v = divergence_gaussian_f32(mean_u, var_u, mean_v, var_v, dx, dy)
            sd = np.sqrt(v)
            for s in range(n_samples):
                z = _vertex_normals(ny * nx, s, seed).reshape(ny, nx).astype(f)
                d = m + f(sd * z)
                for k, c in enumerate(iso.astype(f)):
                    counts[k] += _crossed(d, c)
        else:
            raise ValueError(precision)
        return counts / float(n_samples)
    if mode != "vector":
        raise ValueError(mode)
    if precision == "f64":
        for s in range(n_samples):
            u, v = mc_sample_field(mean_u, var_u, mean_v, var_v, s, seed, first_point)
            d = fd_divergence(u, v, dx, dy)
            for k, c in enumerate(iso):
                counts[k] += _crossed(d, c)
    elif precision == "f32":
        f = np.float32
        mu_u32 = np.asarray(mean_u, f)
        mu_v32 = np.asarray(mean_v, f)
        sd_u32 = np.sqrt(np.asarray(var_u, f))
        sd_v32 = np.sqrt(np.asarray(var_v, f))
        iso32 = iso.astype(f)
        cx_in, cx_bd = f(1.0 / (2.0 * dx)), f(1.0 / dx)
        cy_in, cy_bd = f(1.0 / (2.0 * dy)), f(1.0 / dy)
        for s in range(n_samples):
            zu, zv = _normals(ny * nx, s, seed, first_point)
            u = mu_u32 + sd_u32 * zu.reshape(ny, nx).astype(f)
            v = mu_v32 + sd_v32 * zv.reshape(ny, nx).astype(f)
            ddx = np.empty((ny, nx), f)
            ddx[:, 1:nx - 1] = (u[:, 2:] - u[:, :nx - 2]) * cx_in
            ddx[:, 0] = (u[:, 1] - u[:, 0]) * cx_bd
            ddx[:, nx - 1] = (u[:, nx - 1] - u[:, nx - 2]) * cx_bd
            ddy = np.empty((ny, nx), f)
            ddy[1:ny - 1, :] = (v[2:, :] - v[:ny - 2, :]) * cy_in
            ddy[0, :] = (v[1, :] - v[0, :]) * cy_bd
            ddy[ny - 1, :] = (v[ny - 1, :] - v[ny - 2, :]) * cy_bd
            d = ddx + ddy
            for k, c in enumerate(iso32):
                counts[k] += _crossed(d, c)
    else:
        raise ValueError(precision)
    return counts / float(n_samples)


def mc_lcp_rows(mean_u, var_u, mean_v, var_v, dx: float, dy: float, isovalues,
                n_samples: int, seed: int, j0: int, j1: int, precision: str = "f64"):
    """mc_lcp (vector sampling) on cell rows [j0, j1) of the grid alone: the
    same samples, since every point keeps its Philox counter (its index in
    the whole grid), drawn on point rows j0-1 .. j1+1 (clamped to the grid),
    the rows Eq. 1 reads for vertex rows j0 .. j1.  Equal to
    mc_lcp(...)[:, j0:j1]."""
    ny, nx = np.shape(mean_u)
    a, b = max(0, j0 - 1), min(ny, j1 + 2)
    band = [np.asarray(x)[a:b] for x in (mean_u, var_u, mean_v, var_v)]
    lcp_band = mc_lcp(*band, dx, dy, isovalues, n_samples, seed, precision,
                      first_point=a * nx)
    return lcp_band[:, j0 - a:j1 - a]


def mc_lcp_vertex(div_mean, div_var, isovalues, n_samples: int, seed: int):
    """Vertex-level brute force: draw each vertex divergence independently from
    N(mu, var) with numpy's PCG64 and count crossings.  Converges to lcp() on
    every cell (the closed form's own model), unlike the vector-level MC."""
    rng = np.random.default_rng(seed)
    mu = np.asarray(div_mean, np.float64)
    sd = np.sqrt(np.asarray(div_var, np.float64))
    iso = np.atleast_1d(np.asarray(isovalues, np.float64))
    counts = np.zeros((iso.size,) + (mu.shape[0] - 1, mu.shape[1] - 1), np.int64)
    for _ in range(n_samples):
        d = mu + sd * rng.standard_normal(mu.shape)
        for k, c in enumerate(iso):
            counts[k] += _crossed(d, c)
    return counts / float(n_samples)


# ---------------------------------------------------------------------------
# (e) Isocontour geometry (Section 4, Figs. 1 and 3): the mean-field
#     isocontour of the divergence and the per-member contours of a spaghetti
#     plot, extracted by marching squares.  The paper draws these without
#     stating the extraction; the reading is the textbook algorithm:
#       * a corner is above iff its value >= c (the tie rule of the LCP);
#       * case index = sum of 1, 2, 4, 8 for the corners (i,j), (i+1,j),
#         (i+1,j+1), (i,j+1) that are above;
#       * a crossed edge from corner P (value p) to corner Q (value q) gets
#         the point P + t (Q - P), t = (c - p) / (q - p);
#       * the saddle cases (two opposite corners above) are split by the
#         cell centre value, the mean of the four corners, evaluated in
#         float32 as ((v0 + v1) + (v2 + v3)) / 4 so that both sides take
#         that decision in the same precision.
#     Segments are listed cell by cell in row-major order (j, then i), each
#     as (x0, y0, x1, y1) in grid units (x = i, y = j).
# ---------------------------------------------------------------------------

# edges: 0 bottom (i,j)-(i+1,j), 1 right (i+1,j)-(i+1,j+1),
#        2 top (i,j+1)-(i+1,j+1), 3 left (i,j)-(i,j+1)
_MS_SEGMENTS = {
    0: [], 15: [],
    1: [(3, 0)], 14: [(3, 0)],
    2: [(0, 1)], 13: [(0, 1)],
    4: [(1, 2)], 11: [(1, 2)],
    8: [(2, 3)], 7: [(2, 3)],
    3: [(3, 1)], 12: [(3, 1)],
    6: [(0, 2)], 9: [(0, 2)],
}


def _ms_point(edge, i, j, v00, v10, v11, v01, c):
    if edge == 0:
        return i + (c - v00) / (v10 - v00), float(j)
    if edge == 1:
        return float(i + 1), j + (c - v10) / (v11 - v10)
    if edge == 2:
        return i + (c - v01) / (v11 - v01), float(j + 1)
    return float(i), j + (c - v00) / (v01 - v00)


def marching_squares(field, c: float):
    """Isocontour segments [n][4] float64 of a [ny][nx] field at c."""
    f = np.asarray(field, np.float64)
    ny, nx = f.shape
    segs = []
    for j in range(ny - 1):
        for i in range(nx - 1):
            v00, v10, v11, v01 = f[j, i], f[j, i + 1], f[j + 1, i + 1], f[j + 1, i]
            case = ((v00 >= c) * 1 + (v10 >= c) * 2 + (v11 >= c) * 4 + (v01 >= c) * 8)
            if case in (5, 10):
                f32 = np.float32
                centre = ((f32(v00) + f32(v10)) + (f32(v11) + f32(v01))) * f32(0.25)
                centre_above = bool(centre >= f32(c))
                # centre on the side of corners (i,j) and (i+1,j+1) (case 5)
                # or (i+1,j) and (i,j+1) (case 10): those corners connect
                # through the cell and the contour cuts off the other two
                if (case == 5) == centre_above:
                    pairs = [(0, 1), (2, 3)]
                else:
                    pairs = [(3, 0), (1, 2)]
            else:
                pairs = _MS_SEGMENTS[int(case)]
            for a, b in pairs:
                x0, y0 = _ms_point(a, i, j, v00, v10, v11, v01, c)
                x1, y1 = _ms_point(b, i, j, v00, v10, v11, v01, c)
                segs.append((x0, y0, x1, y1))
    return np.asarray(segs, np.float64).reshape(-1, 4)


def marching_squares_row_counts(field, c: float):
    """Segments per cell row of marching_squares(field, c), from the case
    numbers alone: none for cases 0 and 15 (every corner on one side), two
    for the saddle cases 5 and 10, one for every other case."""
    up = np.asarray(field, np.float64) >= c
    case = (up[:-1, :-1] * 1 + up[:-1, 1:] * 2 + up[1:, 1:] * 4 + up[1:, :-1] * 8)
    n = ((case != 0) & (case != 15)).astype(np.int64) + ((case == 5) | (case == 10))
    return n.sum(axis=1)


def spaghetti(u_members, v_members, dx: float, dy: float, c: float):
    """Per-member isocontours of the divergence (Eq. 1) at c: list of [n][4]."""
    return [marching_squares(fd_divergence(u, v, dx, dy), c)
            for u, v in zip(u_members, v_members)]
