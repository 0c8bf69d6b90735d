"""Plain FP64 oracle of the path extended to 3D vector fields.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

The paper treats 2D fields and names 3D vector fields as future work
(Section 5).  The extension read here changes nothing in the method, only the
dimension:
  * the divergence adds dW/dz to Eq. 1, differenced like the other two axes
    (central inside, first-order one-sided at the boundary), so Eq. 2 and
    Eq. 3 gain a z term of the same form;
  * a cell is a hexahedron with 8 corners, and the level-crossing probability
    of Section 3.1 becomes 1 - prod_8 P(X_k >= c) - prod_8 P(X_k < c), the
    probabilistic marching cubes form of Poethkow et al.

Grid convention: i is the x index, j the y index, k the z index; arrays are
row-major [nz][ny][nx] with x fastest.  U, V, W are the x, y, z components.
Cell (i, j, k) has the corners (i+a, j+b, k+c) for a, b, c in {0, 1}.

Parity status per function:
  divergence_gaussian_3d  pinned (numpy.gradient on the means, closed-form
                          variances at interior, face, edge and corner
                          vertices, linear fields, reduction to the 2D
                          oracle, brute-force sampling)
  divergence_gaussian_3d_f32  pinned to divergence_gaussian_3d: equal where
                          every float32 operation is exact, within float32
                          rounding elsewhere
  lcp_3d                  pinned (marching-cubes limit, i.i.d. closed form,
                          symmetry, range, far isovalues, brute force)
  mc_lcp_3d               pinned statistically against lcp_3d on interior
                          cells; a single draw has no closed form to pin to.
"""

from __future__ import annotations

import numpy as np

from .pdiv_oracle import vertex_probs


def _axis_part(mu, sd, h: float, axis: int):
    """One axis's share of Eq. 2 and Eq. 3 at every vertex: the difference of
    the component along `axis`, central inside (step 2h), first-order
    one-sided at the two boundary planes (step h)."""
    n = mu.shape[axis]
    mean = np.zeros(mu.shape, np.float64)
    var = np.zeros(mu.shape, np.float64)
    for i in range(n):
        if 0 < i < n - 1:
            lo, hi, step = i - 1, i + 1, 2.0 * h
        elif i == 0:
            lo, hi, step = 0, 1, h
        else:
            lo, hi, step = n - 2, n - 1, h
        dst = [slice(None)] * 3
        dst[axis] = i
        src_hi = [slice(None)] * 3
        src_hi[axis] = hi
        src_lo = [slice(None)] * 3
        src_lo[axis] = lo
        dst, src_hi, src_lo = tuple(dst), tuple(src_hi), tuple(src_lo)
        mean[dst] = mu[src_hi] / step - mu[src_lo] / step
        var[dst] = (sd[src_hi] / step) ** 2 + (sd[src_lo] / step) ** 2
    return mean, var


def divergence_gaussian_3d(mean_u, var_u, mean_v, var_v, mean_w, var_w, dx: float, dy: float,
                           dz: float):
    """Mean and variance of the 3D divergence at every vertex, [nz][ny][nx]
    float64 each: the sum over the three axes of Eq. 2 / Eq. 3's terms, the x
    part from U, the y part from V, the z part from W."""
    out_m = None
    out_v = None
    for mu, var, h, axis in ((mean_u, var_u, dx, 2), (mean_v, var_v, dy, 1),
                             (mean_w, var_w, dz, 0)):
        m, v = _axis_part(np.asarray(mu, np.float64), np.sqrt(np.asarray(var, np.float64)),
                          h, axis)
        out_m = m if out_m is None else out_m + m
        out_v = v if out_v is None else out_v + v
    return out_m, out_v


def divergence_gaussian_3d_f32(mean_u, var_u, mean_v, var_v, mean_w, var_w, dx: float,
                               dy: float, dz: float):
    """divergence_gaussian_3d with every operation rounded to float32 in the
    order mean = (mx + my) + mz, var = (vx + vy) + vz, where per axis
    m = (mu_r - mu_l) cm and v = (var_r + var_l) cv, cm = 1/(2h) inside and
    1/h on the two boundary planes, cv = 1/(4h^2) or 1/h^2, each coefficient
    rounded once from float64.  Float32 [nz][ny][nx] planes: the divergence
    Gaussians, bit for bit, of a float32 implementation that rounds in this
    order."""
    f = np.float32
    parts_m, parts_v = [], []
    for mu, var, h, axis in ((mean_u, var_u, dx, 2), (mean_v, var_v, dy, 1),
                             (mean_w, var_w, dz, 0)):
        mu = np.asarray(mu, f)
        var = np.asarray(var, f)
        n = mu.shape[axis]
        i = np.arange(n)
        lo, hi = np.maximum(i - 1, 0), np.minimum(i + 1, n - 1)
        bd = (i == 0) | (i == n - 1)
        shape = [1, 1, 1]
        shape[axis] = n
        cm = np.where(bd, f(1.0 / h), f(1.0 / (2.0 * h))).astype(f).reshape(shape)
        cv = np.where(bd, f(1.0 / (h * h)), f(1.0 / (4.0 * h * h))).astype(f).reshape(shape)
        parts_m.append((np.take(mu, hi, axis) - np.take(mu, lo, axis)) * cm)
        parts_v.append((np.take(var, hi, axis) + np.take(var, lo, axis)) * cv)
    return (parts_m[0] + parts_m[1]) + parts_m[2], (parts_v[0] + parts_v[1]) + parts_v[2]


def fd_divergence_3d(u, v, w, dx: float, dy: float, dz: float):
    """Eq. 1 extended by dW/dz, applied to one deterministic field."""
    zero = np.zeros(np.shape(u), np.float64)
    m, _ = divergence_gaussian_3d(u, zero, v, zero, w, zero, dx, dy, dz)
    return m


def _corners(f):
    """The 8 corner views of every hexahedral cell of a [nz][ny][nx] array."""
    return [f[c:f.shape[0] - 1 + c, b:f.shape[1] - 1 + b, a:f.shape[2] - 1 + a]
            for c in (0, 1) for b in (0, 1) for a in (0, 1)]


def lcp_3d(div_mean, div_var, isovalues):
    """Closed-form LCP maps [K][nz-1][ny-1][nx-1] float64: the probability
    that the c-isosurface passes through a hexahedral cell whose 8 corners
    hold independent Gaussians, 1 - prod P(above) - prod P(below), with the
    >= rule for ties and deterministic corners where the variance is 0."""
    mu = np.asarray(div_mean, np.float64)
    var = np.asarray(div_var, np.float64)
    nz, ny, nx = mu.shape
    iso = np.atleast_1d(np.asarray(isovalues, np.float64))
    out = np.empty((iso.size, nz - 1, ny - 1, nx - 1), np.float64)
    for q, c in enumerate(iso):
        a, b = vertex_probs(mu, var, c)
        all_above = np.ones((nz - 1, ny - 1, nx - 1))
        all_below = np.ones((nz - 1, ny - 1, nx - 1))
        for ca, cb in zip(_corners(a), _corners(b)):
            all_above = all_above * ca
            all_below = all_below * cb
        out[q] = 1.0 - all_above - all_below
    return out


def crossed_3d(d, c: float):
    """Marching-cubes crossing indicator of one deterministic field: the
    corners of a cell are not all on the same side of c (>= is above)."""
    up = [x >= c for x in _corners(np.asarray(d, np.float64))]
    n_up = sum(x.astype(np.int8) for x in up)
    return (n_up != 0) & (n_up != 8)


def mc_lcp_3d(mean_u, var_u, mean_v, var_v, mean_w, var_w, dx: float, dy: float, dz: float,
              isovalues, n_samples: int, seed: int):
    """Vector-level Monte Carlo: draw U, V, W independently at every grid
    point (numpy PCG64), form each sample's divergence by Eq. 1 extended to
    3D, and count per cell how often the isosurface crosses it."""
    rng = np.random.default_rng(seed)
    ms = [np.asarray(x, np.float64) for x in (mean_u, mean_v, mean_w)]
    sds = [np.sqrt(np.asarray(x, np.float64)) for x in (var_u, var_v, var_w)]
    iso = np.atleast_1d(np.asarray(isovalues, np.float64))
    nz, ny, nx = ms[0].shape
    counts = np.zeros((iso.size, nz - 1, ny - 1, nx - 1), np.int64)
    for _ in range(n_samples):
        u, v, w = (m + s * rng.standard_normal(m.shape) for m, s in zip(ms, sds))
        d = fd_divergence_3d(u, v, w, dx, dy, dz)
        for q, c in enumerate(iso):
            counts[q] += crossed_3d(d, c)
    return counts / float(n_samples)


def mc_lcp_3d_vertex(div_mean, div_var, isovalues, n_samples: int, seed: int):
    """Vertex-level brute force: each vertex divergence drawn independently
    from N(mu, var); converges to lcp_3d on every cell."""
    rng = np.random.default_rng(seed)
    mu = np.asarray(div_mean, np.float64)
    sd = np.sqrt(np.asarray(div_var, np.float64))
    iso = np.atleast_1d(np.asarray(isovalues, np.float64))
    nz, ny, nx = mu.shape
    counts = np.zeros((iso.size, nz - 1, ny - 1, nx - 1), np.int64)
    for _ in range(n_samples):
        d = mu + sd * rng.standard_normal(mu.shape)
        for q, c in enumerate(iso):
            counts[q] += crossed_3d(d, c)
    return counts / float(n_samples)
