"""Seeded generators for uncertain 2D vector fields.

Stand-ins for the paper's wind (15 members, 68x68) and Red Sea (20 members,
500x500) ensembles (Section 4), which are not available here.  A field is a
sum of Gaussian-windowed sources/sinks ("radial") and vortices, sampled on the
integer grid x = i, y = j (spacing 1, as in the uniform-grid model of
Section 3).  Per-point spread is drawn independently per component, matching
the independent-Gaussian model of Section 3.

Array convention everywhere: row-major [ny][nx], x (index i) fastest.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 251001190

# Feature truncation radius in widths: beyond 6 w the window factor is
# exp(-18) ~ 1.5e-8 of its peak and is dropped.
_TRUNC = 6.0


@dataclass(frozen=True)
class Feature:
    cx: float
    cy: float
    amp: float
    width: float
    vortex: bool


def gen_features(rng: np.random.Generator, ny: int, nx: int, n: int,
                 amp=(-2.0, 2.0), width=(5.0, 20.0)) -> list[Feature]:
    """n features with centre ~ U[0,nx) x U[0,ny), amplitude ~ U[amp], width ~ U[width],
    kind radial or vortex with probability 1/2 each."""
    cx = rng.uniform(0.0, nx, n)
    cy = rng.uniform(0.0, ny, n)
    a = rng.uniform(amp[0], amp[1], n)
    w = rng.uniform(width[0], width[1], n)
    vort = rng.random(n) < 0.5
    return [Feature(float(cx[k]), float(cy[k]), float(a[k]), float(w[k]), bool(vort[k]))
            for k in range(n)]


def _window(f: Feature, ny: int, nx: int):
    r = _TRUNC * f.width
    x0 = max(0, int(math.floor(f.cx - r)))
    x1 = min(nx, int(math.ceil(f.cx + r)) + 1)
    y0 = max(0, int(math.floor(f.cy - r)))
    y1 = min(ny, int(math.ceil(f.cy + r)) + 1)
    if x0 >= x1 or y0 >= y1:
        return None
    xs = np.arange(x0, x1, dtype=np.float64) - f.cx
    ys = np.arange(y0, y1, dtype=np.float64) - f.cy
    r2 = xs[None, :] ** 2 + ys[:, None] ** 2
    inside = r2 <= (r * r)
    g = np.exp(-r2 / (2.0 * f.width * f.width)) * inside
    return (slice(y0, y1), slice(x0, x1)), xs, ys, r2, g


def mean_field(features, ny: int, nx: int):
    """Smooth velocity field (u, v) in float64 from the features.

    radial: u += A (x-cx)/w g,  v += A (y-cy)/w g   (A>0 source, A<0 sink)
    vortex: u += -A (y-cy)/w g, v += A (x-cx)/w g
    with g = exp(-r^2 / (2 w^2)) and r the distance to the centre."""
    u = np.zeros((ny, nx), np.float64)
    v = np.zeros((ny, nx), np.float64)
    for f in features:
        win = _window(f, ny, nx)
        if win is None:
            continue
        sl, xs, ys, _, g = win
        s = f.amp / f.width
        if f.vortex:
            u[sl] += -s * ys[:, None] * g
            v[sl] += s * xs[None, :] * g
        else:
            u[sl] += s * xs[None, :] * g
            v[sl] += s * ys[:, None] * g
    return u, v


def analytic_divergence(features, ny: int, nx: int):
    """Continuous divergence of mean_field(), from the closed form of each feature.

    A radial feature contributes (A/w) g (2 - r^2/w^2); a vortex contributes 0.
    Used only to pick isovalues at divergence quantiles and to check the
    generator itself; it is the generator's own derivative, not the method."""
    d = np.zeros((ny, nx), np.float64)
    for f in features:
        if f.vortex:
            continue
        win = _window(f, ny, nx)
        if win is None:
            continue
        sl, _, _, r2, g = win
        d[sl] += (f.amp / f.width) * g * (2.0 - r2 / (f.width * f.width))
    return d


def quantile_isovalues(div: np.ndarray, probs) -> np.ndarray:
    """Isovalues at the given quantiles of a divergence map, as float32
    (the precision the GPU path receives them in)."""
    return np.quantile(div.ravel(), np.asarray(probs, np.float64)).astype(np.float32)


def smooth_std_map(rng: np.random.Generator, ny: int, nx: int, lo: float, hi: float,
                   n_bumps: int = 8, width=(100.0, 300.0)) -> np.ndarray:
    """Spread map lo + (hi-lo) s(x,y), s a min-max normalised sum of wide Gaussian bumps."""
    cx = rng.uniform(0.0, nx, n_bumps)
    cy = rng.uniform(0.0, ny, n_bumps)
    w = rng.uniform(width[0], width[1], n_bumps)
    xs = np.arange(nx, dtype=np.float64)
    ys = np.arange(ny, dtype=np.float64)
    s = np.zeros((ny, nx), np.float64)
    for k in range(n_bumps):
        gx = np.exp(-((xs - cx[k]) ** 2) / (2 * w[k] ** 2))
        gy = np.exp(-((ys - cy[k]) ** 2) / (2 * w[k] ** 2))
        s += gy[:, None] * gx[None, :]
    s = (s - s.min()) / max(s.max() - s.min(), 1e-300)
    return lo + (hi - lo) * s


def gen_moments(ny: int, nx: int, seed: int, n_features: int | None = None,
                sigma=(0.05, 0.5), width=(5.0, 20.0)):
    """Independent-Gaussian field in float64: returns dict with mean_u, var_u,
    mean_v, var_v, the features and the analytic divergence of the mean field.
    Spread sigma ~ U[sigma] i.i.d. per point and component; var = sigma^2.
    Default feature count is 6 per 128^2 points (at least 1)."""
    rng = np.random.default_rng(seed)
    if n_features is None:
        n_features = max(1, int(round(6.0 * ny * nx / (128.0 * 128.0))))
    feats = gen_features(rng, ny, nx, n_features, width=width)
    mu, mv = mean_field(feats, ny, nx)
    su = rng.uniform(sigma[0], sigma[1], (ny, nx))
    sv = rng.uniform(sigma[0], sigma[1], (ny, nx))
    return dict(mean_u=mu, var_u=su * su, mean_v=mv, var_v=sv * sv,
                features=feats, ny=ny, nx=nx, dx=1.0, dy=1.0)


def gen_ensemble(ny: int, nx: int, n_members: int, seed: int, n_features: int = 40,
                 std=(0.1, 1.5), dtype=np.float32, width=(5.0, 20.0)):
    """Ensemble members u_m = u_base + su * eps_m, v_m = v_base + sv * eps'_m,
    eps i.i.d. N(0,1), m = 1..M; spread maps su, sv vary smoothly in [std].
    Returns dict with u_members, v_members of shape [M][ny][nx] in dtype, the
    base field, the spread maps and the features."""
    rng = np.random.default_rng(seed)
    feats = gen_features(rng, ny, nx, n_features, width=width)
    ub, vb = mean_field(feats, ny, nx)
    su = smooth_std_map(np.random.default_rng(seed + 1000), ny, nx, std[0], std[1])
    sv = smooth_std_map(np.random.default_rng(seed + 2000), ny, nx, std[0], std[1])
    noise = np.random.default_rng(seed + 3000)
    um = np.empty((n_members, ny, nx), dtype)
    vm = np.empty((n_members, ny, nx), dtype)
    for m in range(n_members):
        um[m] = ub + su * noise.standard_normal((ny, nx))
        vm[m] = vb + sv * noise.standard_normal((ny, nx))
    return dict(u_members=um, v_members=vm, u_base=ub, v_base=vb, std_u=su, std_v=sv,
                features=feats, ny=ny, nx=nx, dx=1.0, dy=1.0, n_members=n_members)


# --------------------------------------------------------------------------
# The five workloads.  C1..C3 follow the sizes of the paper's use (a small
# grid like the wind data, an ensemble fit, a large precision sweep);
# C4 and C5 are the batched and served workloads.
# --------------------------------------------------------------------------

def config_c1():
    """128x128, 6 features, sigma ~ U[0.05,0.5], one isovalue -0.1, MC 2000 samples."""
    f = gen_moments(128, 128, SEED_BASE + 1, n_features=6, sigma=(0.05, 0.5))
    f.update(isovalues=np.array([-0.1], np.float32), n_samples=2000, name="c1_128x128_k1")
    return f


def config_c2(n_members: int = 50):
    """721x1440 ensemble of 50 FP32 members, 40 features of width U[20,100] grid
    units (wide enough to cover the domain), spread in [0.1,1.5]; 8 isovalues
    at divergence quantiles 1/9..8/9; MC 1000 samples."""
    e = gen_ensemble(721, 1440, n_members, SEED_BASE + 2, n_features=40, width=(20.0, 100.0))
    div = analytic_divergence(e["features"], 721, 1440)
    e.update(isovalues=quantile_isovalues(div, np.arange(1, 9) / 9.0), n_samples=1000,
             name="c2_721x1440_m50_k8")
    return e


def config_c3(n: int = 8192):
    """n x n field (default 8192^2), 6 features per 128^2, sigma ~ U[0.01,1.0];
    16 isovalues at divergence quantiles linspace(0.01, 0.99, 16)."""
    f = gen_moments(n, n, SEED_BASE + 3, sigma=(0.01, 1.0))
    div = analytic_divergence(f["features"], n, n)
    f.update(isovalues=quantile_isovalues(div, np.linspace(0.01, 0.99, 16)),
             name=f"c3_{n}x{n}_k16")
    return f


def config_c3_low_spread(n: int = 8192):
    """The precision sweep's field (same seed, so the same features) with a
    small spread, sigma ~ U[0.002, 0.02]: most cells then sit deep in the
    LCP tails (near 0) or are crossed with near certainty (near 1), the cells
    whose accuracy a cancellation-free evaluation must keep.  16 isovalues at
    divergence quantiles linspace(0.01, 0.99, 16)."""
    f = gen_moments(n, n, SEED_BASE + 3, sigma=(0.002, 0.02))
    div = analytic_divergence(f["features"], n, n)
    f.update(isovalues=quantile_isovalues(div, np.linspace(0.01, 0.99, 16)),
             name=f"c3_low_spread_{n}x{n}_k16")
    return f


def batch_sizes(n_fields: int, lo: int, hi: int, seed: int):
    """(ny, nx) pairs with each side round(exp(U[ln lo, ln hi])) independently."""
    rng = np.random.default_rng(seed)
    s = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), (n_fields, 2)))).astype(int)
    return [(int(a), int(b)) for a, b in s]


def config_c4(n_fields: int = 512, lo: int = 64, hi: int = 2048, n_iso: int = 4):
    """Batch of independent fields of uneven size, sigma ~ U[0.05,0.5], with
    n_iso isovalues per field at that field's divergence quantiles."""
    sizes = batch_sizes(n_fields, lo, hi, SEED_BASE + 4)
    probs = np.arange(1, n_iso + 1) / (n_iso + 1.0)
    fields = []
    for k, (ny, nx) in enumerate(sizes):
        f = gen_moments(ny, nx, SEED_BASE + 4 + 7919 * (k + 1), sigma=(0.05, 0.5))
        div = analytic_divergence(f["features"], ny, nx)
        f["isovalues"] = quantile_isovalues(div, probs)
        fields.append(f)
    return fields


def gen_moments_3d(nz: int, ny: int, nx: int, seed: int, sigma=(0.05, 0.5), n_modes: int = 6,
                   dtype=np.float64):
    """Independent-Gaussian 3D field: returns dict with mean_u, var_u, mean_v,
    var_v, mean_w, var_w ([nz][ny][nx] in dtype) and the modes.  Each mean
    component is a sum of n_modes separable waves
        A sin(2 pi kx x/nx + px) sin(2 pi ky y/ny + py) sin(2 pi kz z/nz + pz),
    k ~ U[1, 4] periods per axis, phases U[0, 2 pi), A ~ U[-1, 1] scaled so
    that the component's derivative along its own axis has amplitude |A|
    (sources, sinks and swirls at every scale of the box, with divergences of
    order one).  Spread sigma ~ U[sigma] i.i.d. per point and component."""
    rng = np.random.default_rng(seed)
    n = (nx, ny, nz)
    axes = [np.arange(m, dtype=np.float64) for m in n]  # x, y, z coordinates
    modes = []
    out = {}
    for comp, own in (("u", 0), ("v", 1), ("w", 2)):
        mean = np.zeros((nz, ny, nx), dtype)
        for _ in range(n_modes):
            k = rng.uniform(1.0, 4.0, 3)
            ph = rng.uniform(0.0, 2.0 * math.pi, 3)
            amp = rng.uniform(-1.0, 1.0) * n[own] / (2.0 * math.pi * k[own])
            fx, fy, fz = (np.sin(2.0 * math.pi * k[a] * axes[a] / n[a] + ph[a]) for a in range(3))
            mean += (amp * fz.astype(dtype)[:, None, None]) * (fy.astype(dtype)[None, :, None]
                                                              * fx.astype(dtype)[None, None, :])
            modes.append((comp, amp, tuple(k), tuple(ph)))
        sd = rng.uniform(sigma[0], sigma[1], (nz, ny, nx)).astype(dtype)
        out["mean_" + comp] = mean
        out["var_" + comp] = sd * sd
    out.update(modes=modes, nz=nz, ny=ny, nx=nx)
    return out


def analytic_divergence_3d(modes, nz: int, ny: int, nx: int, step: int = 1):
    """dU/dx + dV/dy + dW/dz of gen_moments_3d's mean field, on every
    step-th point along each axis (for picking isovalues)."""
    n = (nx, ny, nz)
    axes = [np.arange(0, m, step, dtype=np.float64) for m in n]
    div = np.zeros((axes[2].size, axes[1].size, axes[0].size))
    own = {"u": 0, "v": 1, "w": 2}
    for comp, amp, k, ph in modes:
        a0 = own[comp]
        f = []
        for a in range(3):
            arg = 2.0 * math.pi * k[a] * axes[a] / n[a] + ph[a]
            f.append(np.cos(arg) * 2.0 * math.pi * k[a] / n[a] if a == a0 else np.sin(arg))
        div += amp * f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]
    return div


def request_stream(n_requests: int, rate_hz: float, seed: int, frac_new: float = 0.3,
                   side=(256, 4096), n_iso=(1, 4)):
    """Poisson request stream: list of dicts with arrival time (s), kind
    ('new' or 'slider'), side for new square fields, and isovalue count for
    slider requests (uniform in n_iso).  Field choice for sliders is left to
    the caller (uniform over resident fields), given by a uniform draw 'pick'."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n_requests))
    kinds = rng.random(n_requests) < frac_new
    sides = np.rint(np.exp(rng.uniform(math.log(side[0]), math.log(side[1]), n_requests)))
    kiso = rng.integers(n_iso[0], n_iso[1] + 1, n_requests)
    pick = rng.random(n_requests)
    isou = rng.random((n_requests, n_iso[1]))
    out = []
    for r in range(n_requests):
        out.append(dict(t=float(t[r]), kind="new" if kinds[r] else "slider",
                        side=int(sides[r]), n_iso=int(kiso[r]), pick=float(pick[r]),
                        iso_u=isou[r, : int(kiso[r])].copy()))
    return out
