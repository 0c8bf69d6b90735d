"""GPU parity of the closed-form path (moments, Eq. 2-3, LCP, fused) against the
FP64 oracle, through the C ABI.  Oracle inputs are the values the GPU actually
received (storage dtype upcast exactly), so these tests measure the kernels'
float32 arithmetic; the end-to-end storage error is measured at full size in
test_gpu_fullsize.py.  No oracle input comes from a kernel: the divergence
Gaussians given to pdiv_lcp are the oracle's own float32 evaluation of
Eq. 2-3 (which the divergence kernel must reproduce bit for bit)."""

import mpmath
import numpy as np
import pytest
import torch

import oracle as O
import paper_2510_01190_amd as P
import synth
from gpu_util import U32, dev, err_report, host64, moments_dev, stored64

pytestmark = pytest.mark.gpu

LCP_TOL = 1e-5  # absolute LCP error bar for float32 storage


def _field(ny, nx, seed, sigma=(0.05, 0.5)):
    return synth.gen_moments(ny, nx, seed, sigma=sigma)


def _div_tol(mu_u, mu_v, dx, dy):
    # |err(mean)| <= 4u (|a|+|b|) c_x + 4u (|a'|+|b'|) c_y with c = 1/dx on the boundary
    return 8.0 * U32 * (np.abs(mu_u).max() / dx + np.abs(mu_v).max() / dy) + 1e-30


# Widths around the 128-cell strip of the LCP tile (nx - 1 = 127, 128, 129,
# 256, 257) exercise the seam column that lane 63 takes from the seam step.
SHAPES = [(2, 2), (2, 3), (3, 2), (2, 200), (200, 2), (64, 64), (65, 127), (130, 190),
          (97, 4034), (4100, 70), (70, 128), (33, 129), (17, 130), (40, 257), (9, 258)]


# 16-bit storage takes the divergence in 62-column strips (x neighbours from
# the adjacent lanes): widths 62, 63, 124 and 125 put a strip's last output
# column at the right boundary or alone in a strip.
DIV_SHAPES = SHAPES + [(5, 62), (6, 63), (7, 124), (8, 125)]


def _oracle_div(ts, dx=1.0, dy=1.0):
    """The oracle's float32 divergence Gaussians of the stored moments, as
    numpy planes and as device tensors (the pdiv_lcp input of both sides)."""
    rm, rv = O.divergence_gaussian_f32(*stored64(ts), dx, dy)
    return rm, rv, torch.from_numpy(rm).cuda(), torch.from_numpy(rv).cuda()


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", DIV_SHAPES)
def test_divergence_gaussian_parity(shape, dt):
    ny, nx = shape
    f = _field(ny, nx, seed=ny * 1000 + nx)
    dx, dy = 0.75, 1.5
    ts = moments_dev(f, dt)
    dm, dv = P.divergence_gaussian(*ts, dx=dx, dy=dy)
    mu_u, var_u, mu_v, var_v = stored64(ts)
    rm, rv = O.divergence_gaussian(mu_u, var_u, mu_v, var_v, dx, dy)
    gm, gv = host64(dm), host64(dv)
    assert np.max(np.abs(gm - rm)) <= _div_tol(mu_u, mu_v, dx, dy)
    assert np.max(np.abs(gv - rv) / rv) <= 6.0 * U32
    # the kernel rounds in the order the float32 oracle states, bit for bit
    r32m, r32v = O.divergence_gaussian_f32(mu_u, var_u, mu_v, var_v, dx, dy)
    assert np.array_equal(gm, r32m.astype(np.float64))
    assert np.array_equal(gv, r32v.astype(np.float64))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("k", [1, 5, 17])
def test_lcp_parity(shape, k):
    ny, nx = shape
    f = _field(ny, nx, seed=7 + ny + nx)
    ts = moments_dev(f)
    rm, rv, dm, dv = _oracle_div(ts)
    rng = np.random.default_rng(k)
    div = synth.analytic_divergence(f["features"], ny, nx)
    iso = synth.quantile_isovalues(div, rng.uniform(0.02, 0.98, k))
    L = P.lcp(dm, dv, iso)
    ref = O.lcp(rm, rv, iso)
    e = err_report(host64(L), ref)
    assert e["max_abs"] <= LCP_TOL, e
    # the fused kernel gives bitwise the same maps
    Lf = P.lcp_from_moments(*ts, iso)
    assert torch.equal(L, Lf)


@pytest.mark.parametrize("shape", [(65, 129), (40, 258), (130, 190), (3, 2), (33, 128),
                                   (17, 130), (9, 257), (70, 4034)])
def test_pitched_output_equals_dense_and_keeps_padding(shape):
    """Rows padded to a longer pitch hold bitwise the dense maps; the padding
    floats are never written (fused and two-step paths).  Nine isovalues run
    as a chunk of 8, which takes the paired tile when the rows start on
    128-byte lines (streaming stores) and for the fused kernel otherwise too
    (default stores), the split tile for the two-step path on other rows, and
    a chunk of 1 (split tile on these small maps), so this also checks that
    the layouts agree bit for bit, seam column included."""
    ny, nx = shape
    f = _field(ny, nx, seed=5 + nx)
    ts = moments_dev(f)
    iso = np.array([-0.05, -0.02, -0.01, 0.0, 0.004, 0.01, 0.02, 0.03, 0.06], np.float32)
    K = iso.size
    dense = P.lcp_from_moments(*ts, iso)
    rm, rv, dm, dv = _oracle_div(ts)
    for pitch in ((nx - 1 + 31) // 32 * 32, nx + 40):
        for fused in (True, False):
            buf = torch.full((K, ny - 1, pitch), -7.0, device="cuda")
            view = buf[:, :, : nx - 1]
            if fused:
                P.lcp_from_moments(*ts, iso, out=view)
            else:
                P.lcp(dm, dv, iso, out=view)
            torch.cuda.synchronize()
            assert torch.equal(view, dense)
            assert bool((buf[:, :, nx - 1:] == -7.0).all())
    e = P.empty_lcp(K, ny, nx)
    assert e.stride(1) % 32 == 0 and e.stride(1) >= nx - 1
    assert torch.equal(P.lcp_from_moments(*ts, iso, out=e), dense)
    # maps interleaved by rows ([ny-1][K][pitch] buffer), padded and odd pitches
    for pitch in ((nx - 1 + 31) // 32 * 32, nx + 3):
        buf = torch.full((ny - 1, K, pitch), -7.0, device="cuda")
        view = buf.permute(1, 0, 2)[:, :, : nx - 1]
        P.lcp_from_moments(*ts, iso, out=view)
        torch.cuda.synchronize()
        assert torch.equal(view, dense)
        assert bool((buf[:, :, nx - 1:] == -7.0).all())
        P.lcp(dm, dv, iso, out=view)
        assert torch.equal(view, dense)
    assert torch.equal(P.lcp_from_moments(*ts, iso, out=P.empty_lcp(K, ny, nx,
                                                                   interleave_rows=True)), dense)
    ref = O.lcp(rm, rv, iso)
    assert err_report(host64(e), ref)["max_abs"] <= LCP_TOL


def test_pitched_output_views():
    f = _field(20, 40, seed=3)
    ts = moments_dev(f)
    iso = [0.0, 0.1]
    dense = P.lcp_from_moments(*ts, iso)
    # a view that starts one float into its rows is still a valid pitched output
    buf = torch.zeros((2, 19, 64), device="cuda")
    assert torch.equal(P.lcp_from_moments(*ts, iso, out=buf[:, :, 1:40]), dense)
    assert bool((buf[:, :, 0] == 0).all()) and bool((buf[:, :, 40:] == 0).all())
    # maps further apart than their rows need (a gap between maps) are fine
    gap = torch.zeros((2, 20, 64), device="cuda")
    assert torch.equal(P.lcp_from_moments(*ts, iso, out=gap[:, :19, :39]), dense)
    assert bool((gap[:, 19, :] == 0).all())
    with pytest.raises(ValueError):  # cells of a row not contiguous
        P.lcp_from_moments(*ts, iso, out=torch.empty((2, 19, 80), device="cuda")[:, :, :78:2])
    with pytest.raises(P.PdivError):  # maps overlap (the library checks the strides)
        P.lcp_from_moments(*ts, iso, out=torch.empty((20, 50), device="cuda")
                           .as_strided((2, 19, 39), (20, 50, 1)))


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
def test_fused_parity_all_dtypes(dt):
    ny, nx = 257, 300
    f = _field(ny, nx, seed=11, sigma=(0.01, 1.0))
    ts = moments_dev(f, dt)
    iso = np.array([-0.2, -0.01, 0.0, 0.003, 0.05, 0.3], np.float32)
    L = P.lcp_from_moments(*ts, iso, dx=1.0, dy=1.0)
    rm, rv = O.divergence_gaussian(*stored64(ts), 1.0, 1.0)
    ref = O.lcp(rm, rv, iso)
    e = err_report(host64(L), ref)
    assert e["max_abs"] <= LCP_TOL, e


def test_relative_accuracy_near_zero_and_one():
    """Cells with tiny LCP keep their relative accuracy (cancellation-free
    combination); cells near 1 are within a few float32 ulps of 1.  A field
    with small spread puts many cells deep in the tails; a steep ramp of
    divergence means puts cells with one corner confidently on each side."""
    ny, nx = 300, 301
    f = _field(ny, nx, seed=12, sigma=(0.002, 0.02))
    ts = moments_dev(f)
    m, v, dm, dv = _oracle_div(ts)
    div = synth.analytic_divergence(f["features"], ny, nx)
    iso = synth.quantile_isovalues(div, [0.01, 0.3, 0.5, 0.7, 0.99])
    L = host64(P.lcp(dm, dv, iso))
    m, v = m.astype(np.float64), v.astype(np.float64)
    ref = O.lcp(m, v, iso)
    # the FP64 oracle evaluates 1 - A - B literally (absolute error ~1e-16), so
    # it is a relative reference only down to ~1e-9
    small = (ref >= 1e-9) & (ref < 1e-3)
    assert small.sum() > 1000
    rel = np.abs(L[small] - ref[small]) / ref[small]
    assert rel.max() <= 1e-4, rel.max()
    # deeper cells: 40-digit evaluation of the same definition on a sample
    mpmath.mp.dps = 40
    deep = np.argwhere((ref < 1e-9) & (L > 1e-30))
    rng = np.random.default_rng(0)
    for k, j, i in deep[rng.choice(len(deep), min(200, len(deep)), replace=False)]:
        c = mpmath.mpf(float(iso[k]))
        A = mpmath.mpf(1)
        B = mpmath.mpf(1)
        for jj, ii in ((j, i), (j, i + 1), (j + 1, i), (j + 1, i + 1)):
            x = (c - mpmath.mpf(float(m[jj, ii]))) / mpmath.sqrt(2 * mpmath.mpf(float(v[jj, ii])))
            A *= mpmath.erfc(x) / 2
            B *= mpmath.erfc(-x) / 2
        exact = float(1 - A - B)
        assert abs(L[k, j, i] - exact) <= 1e-4 * exact, (k, j, i, L[k, j, i], exact)

    ramp = np.add.outer(np.zeros(40), (np.arange(120) - 60.3) * 0.5).astype(np.float32)
    ramp_v = np.full_like(ramp, 0.01)
    iso2 = np.array([0.1, 1.1, -2.4], np.float32)
    L2 = host64(P.lcp(torch.from_numpy(ramp).cuda(), torch.from_numpy(ramp_v).cuda(), iso2))
    ref2 = O.lcp(ramp.astype(np.float64), ramp_v.astype(np.float64), iso2)
    big = ref2 > 1 - 1e-3
    assert big.sum() >= 3 * 39
    assert np.max(np.abs(L2[big] - ref2[big])) <= 4 * U32


def test_zero_variance_is_exact_crossing_indicator():
    ny, nx = 70, 90
    f = _field(ny, nx, seed=13)
    ts = moments_dev(f)
    m32, _, dm, _ = _oracle_div(ts)
    zero = torch.zeros_like(dm)
    m = m32.astype(np.float64)
    # isovalues equal to vertex means: ties, above by the >= rule
    iso = np.array([m32[5, 5], m32[40, 17], 0.0, 0.01], np.float32)
    L = P.lcp(dm, zero, iso)
    ref = O.lcp(m, np.zeros_like(m), iso)
    assert np.array_equal(host64(L), ref)


def test_mixed_deterministic_corners_and_nan():
    ny, nx = 40, 41
    f = _field(ny, nx, seed=14)
    ts = moments_dev(f)
    m, v, _, _ = _oracle_div(ts)
    v[::3, ::2] = 0.0  # deterministic corners mixed with random ones
    m[20, 20] = np.nan
    iso = np.array([0.0, 0.02], np.float32)
    L = host64(P.lcp(torch.from_numpy(m).cuda(), torch.from_numpy(v).cuda(), iso))
    ref = O.lcp(m.astype(np.float64), v.astype(np.float64), iso)
    nan_ref = np.isnan(ref)
    assert np.array_equal(np.isnan(L), nan_ref) and nan_ref.sum() == 2 * 4
    ok = ~nan_ref
    assert np.max(np.abs(L[ok] - ref[ok])) <= LCP_TOL


def test_far_isovalues_vanish():
    f = _field(50, 60, seed=15)
    ts = moments_dev(f)
    m, v, dm, dv = _oracle_div(ts)
    hi = float(m.max() + 12 * np.sqrt(v.max()))
    lo = float(m.min() - 12 * np.sqrt(v.max()))
    L = host64(P.lcp(dm, dv, [hi, lo]))
    assert L.max() <= 1e-30


def test_many_isovalues_chunking():
    ny, nx = 33, 70
    f = _field(ny, nx, seed=16)
    ts = moments_dev(f)
    iso = np.linspace(-0.3, 0.3, 256).astype(np.float32)
    L = P.lcp_from_moments(*ts, iso)
    ref = O.lcp(*O.divergence_gaussian(*stored64(ts), 1.0, 1.0), iso)
    assert err_report(host64(L), ref)["max_abs"] <= LCP_TOL


# --------------------------------------------------------------------------
# moments
# --------------------------------------------------------------------------

def _moment_tols(x, m):
    # Welford in float32: mean error <= ~2 M u max|x|; variance relative <= ~4 M u
    return 2.0 * m * U32 * np.abs(x).max(), 4.0 * m * U32


@pytest.mark.parametrize("m,shape", [(2, (1, 1)), (3, (5, 7)), (15, (68, 68)), (20, (50, 61)),
                                     (50, (33, 129))])
@pytest.mark.parametrize("ddof", [0, 1])
def test_moments_parity(m, shape, ddof):
    ny, nx = shape
    e = synth.gen_ensemble(ny, nx, m, seed=m + ny, n_features=2, dtype=np.float32)
    u = torch.from_numpy(e["u_members"]).cuda()
    v = torch.from_numpy(e["v_members"]).cuda()
    got = [host64(t) for t in P.moments(u, v, ddof=ddof)]
    ref = O.moments(e["u_members"].astype(np.float64), e["v_members"].astype(np.float64), ddof)
    for g, r, x in ((got[0], ref[0], e["u_members"]), (got[2], ref[2], e["v_members"])):
        ta, _ = _moment_tols(x, m)
        assert np.max(np.abs(g - r)) <= ta
    _, tr = _moment_tols(e["u_members"], m)
    for g, r in ((got[1], ref[1]), (got[3], ref[3])):
        assert np.max(np.abs(g - r) / np.maximum(r, 1e-30)) <= tr + 2 * U32


@pytest.mark.parametrize("in_dt,out_dt", [("f16", "f32"), ("bf16", "f32"), ("f32", "f16"),
                                          ("f32", "bf16")])
def test_moments_dtypes(in_dt, out_dt):
    from gpu_util import TORCH_DT
    m, ny, nx = 20, 30, 45
    e = synth.gen_ensemble(ny, nx, m, seed=3, n_features=2, dtype=np.float32)
    u = torch.from_numpy(e["u_members"]).to(TORCH_DT[in_dt]).cuda()
    v = torch.from_numpy(e["v_members"]).to(TORCH_DT[in_dt]).cuda()
    got = P.moments(u, v, ddof=1, out_dtype=TORCH_DT[out_dt])
    assert all(t.dtype == TORCH_DT[out_dt] for t in got)
    ref = O.moments(host64(u), host64(v), 1)
    # reference rounded to the output dtype exactly as the kernel's store rounds
    for g, r in zip(got, ref):
        rr = host64(torch.from_numpy(r).to(torch.float32).to(TORCH_DT[out_dt]))
        tol = 1e-5 * np.abs(r).max() if out_dt == "f32" else 0.0
        # one output ulp of disagreement is allowed where float32 rounding sits
        # next to a 16-bit rounding boundary
        ulp = np.abs(rr) * (2.0 ** -10 if out_dt == "f16" else 2.0 ** -7)
        if out_dt == "f16":
            ulp = np.maximum(ulp, 2.0 ** -24)  # float16 subnormal spacing
        assert np.all(np.abs(host64(g) - rr) <= np.maximum(tol, ulp) + 1e-30)


def test_moments_member_stride_and_ragged_tail():
    m, ny, nx = 7, 9, 11  # n = 99 points: not a multiple of 4
    rng = np.random.default_rng(5)
    buf = rng.normal(1.0, 0.3, (m, 128)).astype(np.float32)  # stride 128 > 99
    ub = torch.from_numpy(buf).cuda()
    vb = torch.from_numpy(buf[::-1].copy()).cuda()
    outs = [torch.empty((ny, nx), device="cuda") for _ in range(4)]
    L = P.lib()
    import ctypes
    st = L.pdiv_moments(ctypes.c_void_p(ub.data_ptr()), ctypes.c_void_p(vb.data_ptr()), 0, m, ny, nx,
                        128, 1, *[ctypes.c_void_p(o.data_ptr()) for o in outs], 0,
                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    x = buf[:, :99].astype(np.float64).reshape(m, ny, nx)
    y = buf[::-1][:, :99].astype(np.float64).reshape(m, ny, nx)
    ref = O.moments(x, y, 1)
    for g, r in zip(outs, ref):
        assert np.max(np.abs(host64(g) - r)) <= 1e-6 * max(1.0, np.abs(r).max())


def test_pipeline_fit_divergence_lcp():
    """Ensemble -> moments -> fused LCP against the oracle fed with the members."""
    m, ny, nx = 20, 100, 140
    e = synth.gen_ensemble(ny, nx, m, seed=21, n_features=6, dtype=np.float32,
                           width=(10.0, 40.0))
    u = torch.from_numpy(e["u_members"]).cuda()
    v = torch.from_numpy(e["v_members"]).cuda()
    mom = P.moments(u, v, ddof=1)
    div = synth.analytic_divergence(e["features"], ny, nx)
    iso = synth.quantile_isovalues(div, [0.1, 0.5, 0.9])
    L = host64(P.lcp_from_moments(*mom, iso))
    ref = O.lcp(*O.divergence_gaussian(*O.moments(e["u_members"], e["v_members"], 1), 1.0, 1.0),
                iso)
    assert err_report(L, ref)["max_abs"] <= LCP_TOL


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
def test_band_height_does_not_change_the_maps(dt):
    """Every band height gives bitwise the maps of the default choice, for
    dense rows (the LDS-staged paired tile with default stores for the chunk
    of 8 isovalues, the split tile for the chunk of 1) and rows on 128-byte
    lines (the paired tile with streaming stores): bands of 1..7 rows
    exercise the walk's peeled first rows, its odd last row and the ring's
    reuse."""
    ny, nx = 61, 300
    f = _field(ny, nx, seed=77)
    ts = moments_dev(f, dt)
    iso = np.linspace(-0.08, 0.08, 9).astype(np.float32)
    P.set_lcp_band_rows(0)
    dense_ref = P.lcp_from_moments(*ts, iso)
    paired_ref = P.lcp_from_moments(*ts, iso, out=P.empty_lcp(iso.size, ny, nx))
    assert torch.equal(dense_ref, paired_ref)
    try:
        for rows in (1, 2, 3, 4, 5, 6, 7, 13, 64):
            P.set_lcp_band_rows(rows)
            dense = P.lcp_from_moments(*ts, iso)
            paired = P.lcp_from_moments(*ts, iso, out=P.empty_lcp(iso.size, ny, nx))
            torch.cuda.synchronize()
            assert torch.equal(dense, dense_ref), rows
            assert torch.equal(paired, dense_ref), rows
    finally:
        P.set_lcp_band_rows(0)


@pytest.mark.parametrize("shape", [(2, (1 << 20) + 3), ((1 << 17) + 1, 2), (3, 70001)])
@pytest.mark.parametrize("k", [3, 16])
def test_extreme_aspect_ratios(shape, k):
    """One row of a million cells (many strips in one band) and one cell per
    row over 131072 rows (many bands of one strip), dense, padded and
    row-interleaved outputs, against the oracle."""
    ny, nx = shape
    rng = np.random.default_rng(ny + k)
    f = {"mean_u": rng.normal(0, 1, shape), "var_u": rng.uniform(0.01, 0.25, shape),
         "mean_v": rng.normal(0, 1, shape), "var_v": rng.uniform(0.01, 0.25, shape)}
    ts = moments_dev(f)
    iso = np.linspace(-0.8, 0.8, k).astype(np.float32)
    ref = O.lcp(*O.divergence_gaussian(*stored64(ts), 1.0, 1.0), iso)
    for out in (None, P.empty_lcp(k, ny, nx), P.empty_lcp(k, ny, nx, interleave_rows=True)):
        g = host64(P.lcp_from_moments(*ts, iso, out=out))
        assert np.max(np.abs(g - ref)) <= LCP_TOL


def test_band_heights_under_lds_poison():
    """The band-height sweep of the LDS-staged paired tile with every ring
    slot filled with NaN before its row's loads (PDIV_DEBUG_POISON_LDS): a
    read that ran ahead of its load would put NaN in the maps; every band
    height must still give bitwise the maps of the default run."""
    ny, nx = 61, 300
    f = _field(ny, nx, seed=77)
    ts = moments_dev(f, "f32")
    P.set_lcp_band_rows(0)
    for k in (16, 9, 1):
        iso = np.linspace(-0.08, 0.08, k).astype(np.float32)
        ref = P.lcp_from_moments(*ts, iso, out=P.empty_lcp(iso.size, ny, nx))
        torch.cuda.synchronize()
        try:
            P.set_debug(P.DEBUG_POISON_LDS)
            for rows in (0, 1, 2, 3, 4, 5, 6, 7, 13, 64):
                P.set_lcp_band_rows(rows)
                got = P.lcp_from_moments(*ts, iso, out=P.empty_lcp(iso.size, ny, nx))
                torch.cuda.synchronize()
                assert not torch.isnan(got).any(), (k, rows)
                assert torch.equal(got, ref), (k, rows)
        finally:
            P.set_debug(0)
            P.set_lcp_band_rows(0)


# Shapes for the fused kernel's paired tile on rows that start inside a
# 128-byte line: 1, 2, 5, 6 and 9 strips of 128 cells, one and several bands,
# widths whose last strip holds one cell or a full strip.
DENSE_SHAPES = [(40, 130), (61, 300), (99, 701), (70, 642), (33, 1153), (130, 257), (5, 129)]


@pytest.mark.parametrize("shape", DENSE_SHAPES)
@pytest.mark.parametrize("k", [8, 16])
def test_paired_tile_on_unaligned_rows(shape, k):
    """The fused kernel on outputs whose rows start anywhere within a line
    (8-byte stores at any 4-byte offset): planar dense maps, dense maps one
    float into their buffer, planar rows of an odd pitch and maps interleaved
    by rows at an odd pitch -- bitwise the maps of the line-aligned tile,
    nothing written outside the cells, and within 1e-5 of the oracle."""
    ny, nx = shape
    f = _field(ny, nx, seed=13 * nx + ny)
    ts = moments_dev(f)
    iso = np.linspace(-0.06, 0.06, k).astype(np.float32)
    ref = P.lcp_from_moments(*ts, iso, out=P.empty_lcp(k, ny, nx))
    torch.cuda.synchronize()
    cells = (ny - 1) * (nx - 1)
    outs = []
    flat = torch.full((k * cells + 64,), -7.0, device="cuda")
    outs.append((flat, flat[1:1 + k * cells].view(k, ny - 1, nx - 1)))
    outs.append((flat, flat[:k * cells].view(k, ny - 1, nx - 1)))
    for pitch in (nx + 2, nx + 40):
        buf = torch.full((k, ny - 1, pitch), -7.0, device="cuda")
        outs.append((buf, buf[:, :, 3:3 + nx - 1]))
        ibuf = torch.full((ny - 1, k, pitch), -7.0, device="cuda")
        outs.append((ibuf, ibuf.permute(1, 0, 2)[:, :, 1:nx]))
    for buf, view in outs:
        buf.fill_(-7.0)
        P.lcp_from_moments(*ts, iso, out=view)
        torch.cuda.synchronize()
        assert torch.equal(view, ref)
        # every float outside the view keeps the fill
        n_out = int((buf != -7.0).sum())
        assert n_out == k * cells, (n_out, k * cells)
    rm, rv, _, _ = _oracle_div(ts)
    assert err_report(host64(ref), O.lcp(rm, rv, iso))["max_abs"] <= LCP_TOL


def test_unaligned_paired_tile_large_map_and_poison():
    """A map of more than 2^22 cells takes the paired tile on dense rows at
    any isovalue count (here 1 and 4); with the LDS ring poisoned (NaN before
    every row load) and short bands the maps stay bitwise those of the
    line-aligned tile."""
    ny, nx = 2050, 2100
    f = _field(ny, nx, seed=99)
    ts = moments_dev(f)
    for k in (1, 4):
        iso = np.linspace(-0.05, 0.05, k).astype(np.float32)
        ref = P.lcp_from_moments(*ts, iso, out=P.empty_lcp(k, ny, nx))
        torch.cuda.synchronize()
        dense = P.lcp_from_moments(*ts, iso)
        assert torch.equal(dense, ref)
        try:
            P.set_debug(P.DEBUG_POISON_LDS)
            for rows in (0, 1, 3, 7):
                P.set_lcp_band_rows(rows)
                got = P.lcp_from_moments(*ts, iso)
                torch.cuda.synchronize()
                assert not torch.isnan(got).any(), (k, rows)
                assert torch.equal(got, ref), (k, rows)
        finally:
            P.set_debug(0)
            P.set_lcp_band_rows(0)
    # cell rows a..b-1 against the oracle: their vertex rows a..b take Eq. 2-3
    # from rows a-1..b+1, all interior
    a, b = 1000, 1040
    rm, rv = O.divergence_gaussian(*[m[a - 1:b + 2] for m in stored64(ts)], 1.0, 1.0)
    want = O.lcp(rm[1:-1], rv[1:-1], iso)
    assert err_report(host64(dense[:, a:b, :]), want)["max_abs"] <= LCP_TOL


def test_input_checks_reject_bad_values():
    """PDIV_DEBUG_CHECK_INPUTS: a negative variance or a non-finite mean is
    reported as PDIV_ERR_INVALID before any work; admissible inputs pass and
    give the same maps as without the checks."""
    ny, nx = 40, 70
    f = _field(ny, nx, seed=78)
    iso = np.array([0.0, 0.01], np.float32)
    good = moments_dev(f)
    ref = P.lcp_from_moments(*good, iso)
    try:
        P.set_debug(P.DEBUG_CHECK_INPUTS)
        assert torch.equal(P.lcp_from_moments(*good, iso), ref)
        bad_var = [t.clone() for t in good]
        bad_var[3][7, 9] = -1e-3
        bad_mean = [t.clone() for t in good]
        bad_mean[0][3, 5] = float("nan")
        for ts in (bad_var, bad_mean):
            for call in (lambda: P.lcp_from_moments(*ts, iso),
                         lambda: P.divergence_gaussian(*ts),
                         lambda: P.mc_lcp(*ts, iso, n_samples=4, seed=1)):
                with pytest.raises(P.PdivError) as e:
                    call()
                assert e.value.status == 1 and "non-finite" in str(e.value)
        dm, dv = P.divergence_gaussian(*good)
        dv[0, 0] = -1.0
        with pytest.raises(P.PdivError):
            P.lcp(dm, dv, iso)
    finally:
        P.set_debug(0)
