"""GPU parity of the 3D extension (the paper's future work, Section 5)
against the FP64 oracle: the divergence Gaussian with the z term and the
8-corner level-crossing probability, through the C ABI."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2510_01190_amd as P
import synth
from gpu_util import U32, dev, host64

pytestmark = pytest.mark.gpu

KEYS = ("mean_u", "var_u", "mean_v", "var_v", "mean_w", "var_w")
LCP_TOL = 1e-5

# (nz, ny, nx): one cell wide; strips of 63 (dense rows) and 64 cells
# (line-aligned rows) exact and ragged; two bands of 64 rows; layer counts
# that are and are not multiples of the layers a wave carries (4 or 2)
SHAPES = [(2, 2, 2), (3, 5, 70), (9, 33, 130), (17, 40, 64), (5, 3, 127), (4, 130, 65),
          (6, 7, 2), (2, 66, 190), (3, 4, 129)]
SENTINEL = -7.0  # padding floats of an output must keep this


def _padded(k, shape, pitch=None, gap=0):
    """A [k][nz-1][ny-1][nx-1] view with rows padded to `pitch` floats
    (default: the next multiple of 32) and `gap` extra floats between maps,
    filled with SENTINEL; returns (view, backing buffer)."""
    nz, ny, nx = shape
    pitch = pitch or (nx - 1 + 31) // 32 * 32
    map_ = (nz - 1) * (ny - 1) * pitch
    buf = torch.full((k * (map_ + gap),), SENTINEL, dtype=torch.float32, device="cuda")
    view = buf.as_strided((k, nz - 1, ny - 1, nx - 1),
                          (map_ + gap, (ny - 1) * pitch, pitch, 1))
    return view, buf


def _padding_untouched(view, buf):
    mask = torch.ones_like(buf, dtype=torch.bool)
    idx = torch.arange(buf.numel(), device=buf.device).as_strided(view.shape, view.stride())
    mask[idx.reshape(-1)] = False
    return bool(torch.all(buf[mask] == SENTINEL))


def _field(shape, seed, dt="f32", sigma=(0.05, 0.5)):
    f = synth.gen_moments_3d(*shape, seed, sigma=sigma)
    ts = [dev(f[k], dt) for k in KEYS]
    return f, ts


def _axis_means(st, h):
    """The three axis terms of the oracle's mean, each alone (for the
    rounding bound of the float32 sum)."""
    zero = np.zeros_like(st[0])
    parts = []
    for a in range(3):
        args = [zero] * 6
        args[2 * a], args[2 * a + 1] = st[2 * a], st[2 * a + 1]
        parts.append(O.divergence_gaussian_3d(*args, *h)[0])
    return parts


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_divergence_3d_matches_oracle(shape, dt):
    h = (1.0, 0.5, 2.0)
    _, ts = _field(shape, seed=sum(shape), dt=dt)
    dm, dv = P.divergence_gaussian_3d(*ts, *h)
    st = [host64(t) for t in ts]
    rm, rv = O.divergence_gaussian_3d(*st, *h)
    mx, my, mz = _axis_means(st, h)
    # each axis term: a difference, one coefficient and one product rounded;
    # then two additions
    bound_m = 6 * U32 * (np.abs(mx) + np.abs(my) + np.abs(mz)) + 1e-30
    assert np.all(np.abs(host64(dm) - rm) <= bound_m)
    np.testing.assert_allclose(host64(dv), rv, rtol=8 * U32, atol=0)


def _oracle_div3(ts, h=(1.0, 1.0, 1.0)):
    """The oracle's float32 3D divergence Gaussians of the stored volumes, as
    numpy arrays and device tensors: the pdiv_lcp_3d input of both sides."""
    m, v = O.divergence_gaussian_3d_f32(*[host64(t) for t in ts], *h)
    return m, v, torch.from_numpy(m).cuda(), torch.from_numpy(v).cuda()


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_divergence_3d_rounds_like_the_float32_oracle(shape, dt):
    h = (0.75, 1.0, 2.5)
    _, ts = _field(shape, seed=5 * sum(shape), dt=dt)
    dm, dv = P.divergence_gaussian_3d(*ts, *h)
    m, v, _, _ = _oracle_div3(ts, h)
    assert np.array_equal(dm.cpu().numpy(), m) and np.array_equal(dv.cpu().numpy(), v)


@pytest.mark.parametrize("k", [1, 3, 4, 8, 16, 17])
@pytest.mark.parametrize("shape", SHAPES)
def test_lcp_3d_matches_oracle(shape, k):
    _, ts = _field(shape, seed=7 * sum(shape) + k)
    m, v, dm, dv = _oracle_div3(ts)
    m64, v64 = m.astype(np.float64), v.astype(np.float64)
    iso = np.quantile(m64, np.linspace(0.05, 0.95, k)).astype(np.float32)
    g = host64(P.lcp_3d(dm, dv, iso))
    r = O.lcp_3d(m64, v64, iso)
    err = np.abs(g - r)
    print(f"\n[{shape} K={k}] max |LCP - oracle| = {err.max():.3e}, range [{g.min():.9g}, "
          f"{g.max():.9g}]")
    assert err.max() <= LCP_TOL
    assert np.all((g >= 0) & (g <= 1))


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_fused_equals_two_step(shape, dt):
    """pdiv_lcp_3d_from_moments evaluates Eq. 2-3 on the spot with the same
    operands as the divergence kernel: the maps are bitwise the two-step's."""
    h = (1.0, 0.5, 2.0)
    _, ts = _field(shape, seed=3 * sum(shape), dt=dt)
    dm, dv = P.divergence_gaussian_3d(*ts, *h)
    m = _oracle_div3(ts, h)[0]
    for k in (1, 4, 8, 16, 17):
        iso = np.quantile(m, np.linspace(0.05, 0.95, k)).astype(np.float32)
        two = P.lcp_3d(dm, dv, iso)
        fused = P.lcp_3d_from_moments(*ts, iso, *h)
        assert torch.equal(fused, two), (shape, dt, k)


@pytest.mark.parametrize("shape", SHAPES)
def test_line_aligned_layout_is_bitwise_the_dense_maps(shape):
    """Rows padded to whole 128-byte lines take the 64-cell tile with the
    seam step; the maps are bitwise those of the dense layout (63-cell
    tile), which the oracle test above checks, and the padding is never
    written.  Pitches of 32 (line-aligned) and of nx - 1 + 5 (not aligned),
    with and without a gap between maps."""
    _, ts = _field(shape, seed=11 * sum(shape))
    m, _, dm, dv = _oracle_div3(ts)
    nz, ny, nx = shape
    for k in (1, 2, 3, 4, 8, 16, 17):
        iso = np.quantile(m, np.linspace(0.05, 0.95, k)).astype(np.float32)
        dense = P.lcp_3d(dm, dv, iso)
        for pitch, gap in ((None, 0), (None, 64), ((nx - 1 + 31) // 32 * 32 + 32, 32),
                           (nx - 1 + 5, 3)):
            view, buf = _padded(k, shape, pitch, gap)
            P.lcp_3d(dm, dv, iso, out=view)
            assert torch.equal(view, dense), (shape, k, pitch, gap)
            assert _padding_untouched(view, buf), (shape, k, pitch, gap)


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_fused_line_aligned_layout_equals_two_step(shape, dt):
    h = (0.5, 1.0, 1.5)
    _, ts = _field(shape, seed=13 * sum(shape), dt=dt)
    dm, dv = P.divergence_gaussian_3d(*ts, *h)
    m = _oracle_div3(ts, h)[0]
    for k in (1, 4, 8, 16):
        iso = np.quantile(m, np.linspace(0.05, 0.95, k)).astype(np.float32)
        two = P.lcp_3d(dm, dv, iso)
        view, buf = _padded(k, shape)
        P.lcp_3d_from_moments(*ts, iso, *h, out=view)
        assert torch.equal(view, two), (shape, dt, k)
        assert _padding_untouched(view, buf)


def test_empty_lcp_3d_pads_rows_to_lines():
    shape = (4, 9, 100)
    _, ts = _field(shape, seed=17)
    _, _, dm, dv = _oracle_div3(ts)
    out = P.empty_lcp_3d(3, *shape)
    assert out.stride() == (3 * 8 * 128, 8 * 128, 128, 1) and out.data_ptr() % 128 == 0
    iso = [-0.1, 0.0, 0.1]
    assert torch.equal(P.lcp_3d(dm, dv, iso, out=out), P.lcp_3d(dm, dv, iso))


def test_lcp_3d_end_to_end_float32():
    """From the float64 field through float32 storage and arithmetic."""
    shape = (9, 33, 130)
    f, ts = _field(shape, seed=99)
    iso = np.linspace(-0.6, 0.6, 5).astype(np.float32)
    g = host64(P.lcp_3d(*P.divergence_gaussian_3d(*ts), iso))
    r = O.lcp_3d(*O.divergence_gaussian_3d(*[f[k] for k in KEYS], 1.0, 1.0, 1.0), iso)
    err = float(np.max(np.abs(g - r)))
    print(f"\n[end to end] max |LCP - oracle(float64 field)| = {err:.3e}")
    assert err <= LCP_TOL


def test_zero_variance_is_marching_cubes():
    shape = (6, 20, 70)
    f = synth.gen_moments_3d(*shape, 5)
    ts = [dev(f[k] if k.startswith("mean") else 0.0 * f[k]) for k in KEYS]
    m32, v32, dm, dv = _oracle_div3(ts)
    assert float(np.abs(v32).max()) == 0.0
    m64 = m32.astype(np.float64)
    iso = np.quantile(m64, [0.1, 0.5, 0.9]).astype(np.float32)
    iso[1] = m32[3, 10, 35]  # a tie at a vertex: >= counts as above
    g = host64(P.lcp_3d(dm, dv, iso))
    for q, c in enumerate(iso):
        np.testing.assert_array_equal(g[q], O.crossed_3d(m64, float(c)).astype(np.float64))


def test_nan_reaches_exactly_its_cells():
    shape = (5, 9, 70)
    _, ts = _field(shape, seed=3)
    _, _, dm, dv = _oracle_div3(ts)
    dm[2, 4, 66] = float("nan")
    g = host64(P.lcp_3d(dm, dv, [0.0, 0.3]))
    bad = np.zeros(g.shape[1:], bool)
    bad[1:3, 3:5, 65:67] = True
    assert np.all(np.isnan(g[:, bad]))
    assert not np.any(np.isnan(g[:, ~bad]))


def test_bench_size_sampled_slabs():
    """The benchmark's 3D workload (512^3, float32, 4 isovalues): every cell
    in [0, 1] and finite, and slabs of cell layers at the bottom, middle and
    top of the volume against the oracle."""
    n = 512
    f = synth.gen_moments_3d(n, n, n, synth.SEED_BASE + 30, dtype=np.float32)
    ts = [torch.from_numpy(f[k]).cuda() for k in KEYS]

    def oracle_vertices(k0):
        # vertex planes k0..k0+2 from the z slab around them (planes k0-1 ..
        # k0+3): inside the slab they are differenced as in the whole volume
        a, b = max(0, k0 - 1), min(n, k0 + 4)
        m, v = O.divergence_gaussian_3d(*[f[k][a:b].astype(np.float64) for k in KEYS],
                                        1.0, 1.0, 1.0)
        return m[k0 - a:k0 - a + 3], v[k0 - a:k0 - a + 3]

    iso = np.quantile(oracle_vertices(n // 2 - 2)[0], [0.2, 0.4, 0.6, 0.8]).astype(np.float32)
    dm, dv = P.divergence_gaussian_3d(*ts)
    out = P.lcp_3d(dm, dv, iso)
    assert torch.equal(P.lcp_3d_from_moments(*ts, iso), out)
    # the benchmark's layouts: rows padded to 512 floats, two-step and fused
    padded = P.empty_lcp_3d(4, n, n, n)
    assert torch.equal(P.lcp_3d(dm, dv, iso, out=padded), out)
    assert torch.equal(P.lcp_3d_from_moments(*ts, iso, out=padded), out)
    del padded
    assert not torch.isnan(out).any()
    assert float(out.min()) >= 0.0 and float(out.max()) <= 1.0
    worst = 0.0
    for k0 in (0, n // 2 - 2, n - 3):
        r = O.lcp_3d(*oracle_vertices(k0), iso)
        worst = max(worst, float(np.max(np.abs(host64(out[:, k0:k0 + 2]) - r))))
    print(f"\n[512^3 K=4] max |LCP - oracle(stored volumes)| on sampled slabs = {worst:.3e}")
    assert worst <= LCP_TOL
