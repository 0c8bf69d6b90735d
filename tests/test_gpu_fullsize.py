"""Parity at the full workload sizes, in the launch configuration the benchmark
times, on sampled rows the oracle computes band by band.

8192x8192, 16 isovalues (the precision sweep): float32 storage must be within
1e-5 of the FP64 oracle on the stored values and on the original float64
field; float16 / bfloat16 errors are measured and stated.  721x1440 with 50
members (the ensemble pipeline): fit -> fused LCP against the oracle run on
the same members.  The Monte Carlo comparison at 8192x8192, 16 isovalues and
1000 samples (and on the ensemble at 8 isovalues): crossing counts on sampled
rows against the oracle's float32 MC, drawn from the same Philox counters.
The other benchmark launches at their sizes: the 8192x8192 mean-field
isocontour and the 50-member spaghetti plot (every row's segment count and
sampled rows' segments against the oracle), the 512-field batch (autotuned,
graph-replayed) and the served stream's fields up to 4096^2 (sampled fields
and rows within 1e-5 of the oracle)."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2510_01190_amd as P
import synth
from gpu_util import TORCH_DT, U32, host64

pytestmark = pytest.mark.gpu

LCP_TOL = 1e-5


def oracle_rows(mom, dx, dy, iso, j0, j1):
    """Oracle LCP on cell rows [j0, j1) of the full grid: vertex rows j0..j1
    need moment rows j0-1 .. j1+1; the band's own edge rows are interior rows
    of the full grid unless they are its true boundary."""
    ny = mom[0].shape[0]
    a, b = max(0, j0 - 1), min(ny, j1 + 2)
    m, v = O.divergence_gaussian(*[x[a:b] for x in mom], dx, dy)
    return O.lcp(m[j0 - a:j1 + 1 - a], v[j0 - a:j1 + 1 - a], iso)


@pytest.fixture(scope="module")
def c3():
    return synth.config_c3()


ROWS = [(0, 6), (1, 3), (4095, 4101), (8185, 8191)]


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
def test_c3_sampled_rows(c3, dt):
    ny, nx = c3["ny"], c3["nx"]
    iso = c3["isovalues"]
    ts = [torch.from_numpy(c3[k]).to(TORCH_DT[dt]).cuda() for k in
          ("mean_u", "var_u", "mean_v", "var_v")]
    # the benchmark's launch: rows padded to a 128-byte multiple (pitch 8192),
    # the 16 maps' rows j adjacent in memory
    out = P.lcp_from_moments(*ts, iso, out=P.empty_lcp(iso.size, ny, nx, interleave_rows=True))
    assert out.stride(2) == 1 and out.stride(0) == 8192 and out.stride(1) == 8192 * iso.size
    torch.cuda.synchronize()
    stored = None
    worst_k, worst_e = 0.0, 0.0
    for j0, j1 in ROWS:
        g = host64(out[:, j0:j1, :])
        if stored is None:
            stored = [host64(t) for t in ts]
        ref_k = oracle_rows(stored, 1.0, 1.0, iso, j0, j1)          # kernel arithmetic
        ref_e = oracle_rows([c3[k] for k in ("mean_u", "var_u", "mean_v", "var_v")],
                            1.0, 1.0, iso, j0, j1)                   # end to end
        worst_k = max(worst_k, float(np.max(np.abs(g - ref_k))))
        worst_e = max(worst_e, float(np.max(np.abs(g - ref_e))))
    print(f"\n[c3 {dt}] max |LCP - oracle(stored)| = {worst_k:.3e}, "
          f"max |LCP - oracle(float64 field)| = {worst_e:.3e}")
    assert worst_k <= LCP_TOL
    if dt == "f32":
        assert worst_e <= LCP_TOL
    del out, ts
    torch.cuda.empty_cache()


MC_ROWS = [(0, 2), (4095, 4097), (8189, 8191)]


def test_c3_mc_sampled_rows(c3):
    """The Monte Carlo comparison at its benchmark launch (the whole 8192x8192
    field, 16 isovalues, 1000 samples, seed 2025) against the oracle's
    float32-precision MC on bottom, middle and top cell rows: each point keeps
    its Philox counter, so the oracle's band draws the kernel's samples."""
    ny, nx = c3["ny"], c3["nx"]
    iso = c3["isovalues"]
    S, seed = 1000, 2025
    ts = [torch.from_numpy(c3[k]).float().cuda() for k in ("mean_u", "var_u", "mean_v", "var_v")]
    out = torch.empty((iso.size, ny - 1, nx - 1), device="cuda")
    P.mc_lcp(*ts, iso, n_samples=S, seed=seed, out=out)
    torch.cuda.synchronize()
    stored = [host64(t) for t in ts]
    total, n = 0, 0
    for j0, j1 in MC_ROWS:
        g = host64(out[:, j0:j1, :])
        r = O.mc_lcp_rows(*stored, 1.0, 1.0, iso, S, seed, j0, j1, precision="f32")
        flips = np.abs(np.rint(g * S) - np.rint(r * S))
        total += int(flips.sum())
        n += flips.size
    print(f"\n[c3 mc S={S}] {total} crossing-count flips over {n} cells x {S} samples")
    assert total <= 5 + 1e-5 * n * S
    del out, ts
    torch.cuda.empty_cache()


def test_c3_properties_whole_grid(c3):
    """Properties that hold at any size, checked on every cell: range [0,1],
    no NaN, the two-step path equals the fused path bitwise, and the pitched
    planar and row-interleaved (benchmark) layouts hold the same maps as the
    dense one."""
    ts = [torch.from_numpy(c3[k]).float().cuda() for k in ("mean_u", "var_u", "mean_v", "var_v")]
    iso = c3["isovalues"][[0, 7, 15]]
    fused = P.lcp_from_moments(*ts, iso)
    dm, dv = P.divergence_gaussian(*ts)
    two = P.lcp(dm, dv, iso)
    assert torch.equal(fused, two)
    ny, nx = ts[0].shape
    for inter in (False, True):
        pitched = P.lcp_from_moments(*ts, iso, out=P.empty_lcp(iso.size, ny, nx,
                                                              interleave_rows=inter))
        assert torch.equal(fused, pitched)
        del pitched
    assert not torch.isnan(fused).any()
    assert float(fused.min()) >= 0.0 and float(fused.max()) <= 1.0
    del fused, two, dm, dv, ts
    torch.cuda.empty_cache()


def test_c2_pipeline_full_size():
    e = synth.config_c2()
    u = torch.from_numpy(e["u_members"]).cuda()
    v = torch.from_numpy(e["v_members"]).cuda()
    mom = P.moments(u, v, ddof=1)
    out = P.lcp_from_moments(*mom, e["isovalues"])
    torch.cuda.synchronize()
    ref_mom = O.moments(e["u_members"][:, :40], e["v_members"][:, :40], 1)
    for g, r in zip(mom, ref_mom):
        assert np.max(np.abs(host64(g)[:40] - r)) <= 2e-5 * max(1.0, np.abs(r).max())
    for j0, j1 in [(0, 3), (360, 364), (717, 720)]:
        a, b = max(0, j0 - 1), min(721, j1 + 2)
        rm = O.moments(e["u_members"][:, a:b], e["v_members"][:, a:b], 1)
        m, vv = O.divergence_gaussian(*rm, 1.0, 1.0)
        ref = O.lcp(m[j0 - a:j1 + 1 - a], vv[j0 - a:j1 + 1 - a], e["isovalues"])
        assert np.max(np.abs(host64(out[:, j0:j1, :]) - ref)) <= LCP_TOL


# --------------------------------------------------------------------------
# Near-0 and near-1 cells on the kernel the benchmark times: the fused path
# with 16 isovalues into rows padded to 128-byte lines and interleaved by
# isovalue (the paired tile with its rows staged through LDS), on a
# low-spread field whose cells sit deep in the LCP tails or are crossed with
# near certainty.  The oracle's input is its own float32 evaluation of
# Eq. 2-3 on the stored values (what the kernel holds, bit for bit), so the
# comparison isolates the LCP arithmetic, whose relative accuracy near 0 and
# absolute accuracy near 1 the cancellation-free combination must keep.
# --------------------------------------------------------------------------

def _near01_check(g, m32, v32, iso, rng, n_deep=60):
    """Assertions of the near-0/1 test on one band; returns bin counts."""
    import mpmath
    m, v = m32.astype(np.float64), v32.astype(np.float64)
    ref = O.lcp(m, v, iso)
    assert np.max(np.abs(g - ref)) <= LCP_TOL
    # relative accuracy down to 1e-9, where the float64 oracle's literal
    # 1 - A - B is still a relative reference
    small = (ref >= 1e-9) & (ref < 1e-3)
    rel = np.abs(g[small] - ref[small]) / ref[small]
    assert rel.size == 0 or rel.max() <= 1e-4, rel.max()
    # deeper cells: 40-digit evaluation of the definition on a sample
    mpmath.mp.dps = 40
    deep = np.argwhere((ref < 1e-9) & (g > 1e-30))
    for k, j, i in deep[rng.choice(len(deep), min(n_deep, len(deep)), replace=False)]:
        c = mpmath.mpf(float(iso[k]))
        A = mpmath.mpf(1)
        B = mpmath.mpf(1)
        for jj, ii in ((j, i), (j, i + 1), (j + 1, i), (j + 1, i + 1)):
            x = (c - mpmath.mpf(float(m[jj, ii]))) / mpmath.sqrt(2 * mpmath.mpf(float(v[jj, ii])))
            A *= mpmath.erfc(x) / 2
            B *= mpmath.erfc(-x) / 2
        exact = float(1 - A - B)
        assert abs(g[k, j, i] - exact) <= 1e-4 * exact, (k, j, i, g[k, j, i], exact)
    # near 1: within a few float32 ulps
    big = ref > 1 - 1e-3
    if big.any():
        assert np.max(np.abs(g[big] - ref[big])) <= 4 * U32
    return int(small.sum()), len(deep), int(big.sum())


def test_near_zero_and_one_whole_2048_grid():
    f = synth.config_c3_low_spread(2048)
    iso = f["isovalues"]
    keys = ("mean_u", "var_u", "mean_v", "var_v")
    ts = [torch.from_numpy(f[k]).float().cuda() for k in keys]
    out = P.lcp_from_moments(*ts, iso, out=P.empty_lcp(16, 2048, 2048, interleave_rows=True))
    m32, v32 = O.divergence_gaussian_f32(*[host64(t) for t in ts], 1.0, 1.0)
    g = host64(out)
    n_small, n_deep, n_big = _near01_check(g, m32, v32, iso, np.random.default_rng(1),
                                           n_deep=200)
    print(f"\n[2048^2 low spread] cells in [1e-9,1e-3): {n_small}, < 1e-9: {n_deep}, "
          f"> 1-1e-3: {n_big}")
    assert n_small > 10000 and n_deep > 10000 and n_big > 1000


@pytest.fixture(scope="module")
def c3_low():
    return synth.config_c3_low_spread()


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
def test_near_zero_and_one_8192_sampled_rows(c3_low, dt):
    ny, nx = c3_low["ny"], c3_low["nx"]
    iso = c3_low["isovalues"]
    keys = ("mean_u", "var_u", "mean_v", "var_v")
    ts = [torch.from_numpy(c3_low[k]).to(TORCH_DT[dt]).cuda() for k in keys]
    out = P.lcp_from_moments(*ts, iso, out=P.empty_lcp(iso.size, ny, nx, interleave_rows=True))
    assert out.stride(0) == 8192 and out.stride(1) == 8192 * iso.size
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    totals = np.zeros(3, np.int64)
    for j0, j1 in [(0, 40), (4090, 4154), (8150, 8191)]:
        a, b = max(0, j0 - 1), min(ny, j1 + 2)
        m32, v32 = O.divergence_gaussian_f32(*[host64(t[a:b]) for t in ts], 1.0, 1.0)
        sl = slice(j0 - a, j1 + 1 - a)
        totals += _near01_check(host64(out[:, j0:j1, :]), m32[sl], v32[sl], iso, rng)
    print(f"\n[8192^2 low spread {dt}] cells in [1e-9,1e-3): {totals[0]}, < 1e-9: {totals[1]}, "
          f"> 1-1e-3: {totals[2]}")
    assert totals[0] > 10000 and totals[1] > 10000 and totals[2] > 100
    del out, ts
    torch.cuda.empty_cache()


# --- the other benchmark launches at their full sizes ------------------------

def _oracle_segments(field32, c, j0, j1):
    """Oracle segments of cell rows [j0, j1) of a float32 field, in the whole
    field's coordinates (a cell row's segments depend on its two vertex rows
    alone)."""
    r = O.marching_squares(field32[j0:j1 + 1].astype(np.float64), float(np.float32(c)))
    r[:, [1, 3]] += j0
    return r


def _segments_in_rows(s, o):
    """Every segment lies in the cell row its offsets give it, inside the
    grid, with both endpoints on cell edges (an integral x or y)."""
    rows = np.repeat(np.arange(o.size - 1), np.diff(o))
    lo = np.minimum(s[:, 1], s[:, 3])
    hi = np.maximum(s[:, 1], s[:, 3])
    assert np.all(lo >= rows) and np.all(hi <= rows + 1)
    for a, b in ((0, 1), (2, 3)):
        assert np.all((s[:, a] == np.floor(s[:, a])) | (s[:, b] == np.floor(s[:, b])))


CONTOUR_ROWS = [(0, 3), (1021, 1024), (4095, 4098), (6143, 6146), (8188, 8191)]


def test_c3_isocontour_full_size(c3):
    """The mean-field isocontour of the 8192x8192 field at its middle
    isovalue (the benchmark's contour launch: count, row scan, write).  The
    float32 divergence mean the oracle computes from the stored moments is the
    field both sides contour.  Every row's segment count equals the oracle's;
    the segments of sampled rows match the oracle's one to one; every segment
    lies on cell edges in its own row."""
    ny, nx = c3["ny"], c3["nx"]
    c = float(c3["isovalues"][c3["isovalues"].size // 2])
    m32 = [c3[k].astype(np.float32) for k in ("mean_u", "var_u", "mean_v", "var_v")]
    d32 = O.divergence_gaussian_f32(*m32, 1.0, 1.0)[0]
    del m32
    field = torch.from_numpy(d32).cuda()
    offs = torch.empty(ny, dtype=torch.int64, device="cuda")
    L = P.lib()
    assert L.pdiv_isocontour(P._p(field.data_ptr()), ny, nx, c, P._p(offs.data_ptr()), None, 0,
                             P._stream()) == 0
    n = int(offs[-1].item())
    segs = torch.empty((n, 4), device="cuda")
    assert L.pdiv_isocontour(P._p(field.data_ptr()), ny, nx, c, P._p(offs.data_ptr()),
                             P._p(segs.data_ptr()), n, P._stream()) == 0
    torch.cuda.synchronize()
    o = offs.cpu().numpy()
    s = host64(segs)
    assert o[0] == 0 and o[-1] == n == len(s)
    np.testing.assert_array_equal(np.diff(o), O.marching_squares_row_counts(d32, np.float32(c)))
    _segments_in_rows(s, o)
    for j0, j1 in CONTOUR_ROWS:
        r = _oracle_segments(d32, c, j0, j1)
        g = s[o[j0]:o[j1]]
        assert g.shape == r.shape
        assert np.all(np.abs(g - r) <= 4 * U32 * (1 + np.abs(r)))
    print(f"\n[c3 isocontour] {n} segments, every row's count equal to the oracle's")
    del field, segs, offs
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def c2():
    e = synth.config_c2()
    e["mom32"] = [m.astype(np.float32) for m in O.moments(e["u_members"], e["v_members"], 1)]
    return e


def test_c2_mc_sampled_rows(c2):
    """The Monte Carlo of the Fig. 4 curve at its largest sample count (the
    fitted 721x1440 ensemble, 8 isovalues, 1000 samples, seed 2025) against
    the oracle's float32-decision MC on bottom, middle and top cell rows; the
    fit is the oracle's, stored as float32."""
    ts = [torch.from_numpy(m).cuda() for m in c2["mom32"]]
    iso = c2["isovalues"]
    S, seed = 1000, 2025
    out = torch.empty((iso.size, 720, 1439), device="cuda")
    P.mc_lcp(*ts, iso, n_samples=S, seed=seed, out=out)
    torch.cuda.synchronize()
    stored = [m.astype(np.float64) for m in c2["mom32"]]
    total, n = 0, 0
    for j0, j1 in [(0, 2), (359, 361), (718, 720)]:
        g = host64(out[:, j0:j1, :])
        r = O.mc_lcp_rows(*stored, 1.0, 1.0, iso, S, seed, j0, j1, precision="f32")
        flips = np.abs(np.rint(g * S) - np.rint(r * S))
        total += int(flips.sum())
        n += flips.size
    print(f"\n[c2 mc S={S}] {total} crossing-count flips over {n} cells x {S} samples")
    assert total <= 5 + 1e-5 * n * S


def test_c2_spaghetti_full_size(c2):
    """The spaghetti plot of the 50-member 721x1440 ensemble at the middle
    isovalue (the benchmark's call): per member, every row's segment count
    equals the oracle's on that member's float32 divergence (Eq. 1), and
    sampled rows match the oracle's segments one to one."""
    m, ny, nx = c2["u_members"].shape
    u = torch.from_numpy(c2["u_members"]).cuda()
    v = torch.from_numpy(c2["v_members"]).cuda()
    c = float(np.float32(c2["isovalues"][4]))
    work = torch.empty((m, ny, nx), device="cuda")
    offs = torch.empty(m * (ny - 1) + 1, dtype=torch.int64, device="cuda")
    L = P.lib()
    args = (P._p(u.data_ptr()), P._p(v.data_ptr()), 0, m, ny, nx, 0, 1.0, 1.0, c,
            P._p(work.data_ptr()), P._p(offs.data_ptr()))
    assert L.pdiv_spaghetti(*args, None, 0, P._stream()) == 0
    n = int(offs[-1].item())
    segs = torch.empty((n, 4), device="cuda")
    assert L.pdiv_spaghetti(*args, P._p(segs.data_ptr()), n, P._stream()) == 0
    torch.cuda.synchronize()
    o = offs.cpu().numpy()
    s = host64(segs)
    assert o[0] == 0 and o[-1] == n
    z = np.zeros((ny, nx))
    for q in range(m):
        oq = o[q * (ny - 1):(q + 1) * (ny - 1) + 1]
        sq = s[oq[0]:oq[-1]]
        d32 = O.divergence_gaussian_f32(c2["u_members"][q].astype(np.float64), z,
                                        c2["v_members"][q].astype(np.float64), z, 1.0, 1.0)[0]
        np.testing.assert_array_equal(np.diff(oq), O.marching_squares_row_counts(d32, c))
        _segments_in_rows(sq, oq - oq[0])
        for j0, j1 in [(0, 2), (359, 361), (718, 720)]:
            r = _oracle_segments(d32, c, j0, j1)
            g = s[oq[j0]:oq[j1]]
            assert g.shape == r.shape
            assert np.all(np.abs(g - r) <= 4 * U32 * (1 + np.abs(r)))
    print(f"\n[c2 spaghetti] {n} segments over {m} members")
    del u, v, work, segs, offs
    torch.cuda.empty_cache()


def test_c4_batch_full_size(tmp_path, monkeypatch):
    """The 512 fields of uneven size (sides log-uniform in [64, 2048], 4
    isovalues each) in the benchmark's launch: one persistent launch, tile
    chosen by the autotuner, replayed as a graph.  Every field's maps equal
    its own fused launch bitwise; sampled fields (the largest, the smallest
    and seeded others) are within 1e-5 of the FP64 oracle, whole for small
    fields and on bottom, middle and top rows for large ones."""
    monkeypatch.setenv("PDIV_TUNE_CACHE", str(tmp_path / "tune.json"))
    F = synth.config_c4()
    fields = []
    for f in F:
        d = {k: torch.from_numpy(f[k]).float().cuda() for k in ("mean_u", "var_u", "mean_v", "var_v")}
        d["isovalues"] = torch.from_numpy(f["isovalues"]).cuda()
        fields.append(d)
    b = P.Batch(fields, graph=True, autotune=True)
    b.launch()
    b.launch()
    torch.cuda.synchronize()
    for f, g in zip(F, b.fields):
        alone = P.lcp_from_moments(g["mean_u"], g["var_u"], g["mean_v"], g["var_v"],
                                   f["isovalues"], out=P.empty_lcp(4, f["ny"], f["nx"]))
        assert torch.equal(alone, g["lcp"])
    cells = np.array([(f["ny"] - 1) * (f["nx"] - 1) for f in F])
    order = np.argsort(cells)
    rng = np.random.default_rng(4)
    pick = sorted(set(order[:3].tolist() + order[-3:].tolist() +
                      rng.choice(len(F), 10, replace=False).tolist()))
    worst = 0.0
    for i in pick:
        f, g = F[i], b.fields[i]
        mom = [f[k].astype(np.float32).astype(np.float64)
               for k in ("mean_u", "var_u", "mean_v", "var_v")]
        ny = f["ny"]
        bands = [(0, ny - 1)] if cells[i] <= 250_000 else \
            [(0, 2), (ny // 2, ny // 2 + 2), (ny - 3, ny - 1)]
        for j0, j1 in bands:
            ref = oracle_rows(mom, 1.0, 1.0, f["isovalues"], j0, j1)
            worst = max(worst, float(np.max(np.abs(host64(g["lcp"][:, j0:j1, :]) - ref))))
    print(f"\n[c4 batch] {b.info()}; max |LCP - oracle| over {len(pick)} fields = {worst:.3e}")
    assert worst <= LCP_TOL
    b.close()
    del fields, b
    torch.cuda.empty_cache()


def test_c5_served_full_size():
    """The served stream's fields at their full sizes (new fields of sides
    256 to 4096 cut from one 4096^2 field, as the benchmark does; 24 GiB
    budget, two streams, pinned staging set aside): slider requests of 1-4
    isovalues submitted while the uploads run, each within 1e-5 of the FP64
    oracle on the stored host planes (whole for small fields, sampled rows for
    large ones)."""
    big_side = 4096
    f = synth.gen_moments(big_side, big_side, synth.SEED_BASE + 5 + big_side,
                          n_features=big_side * big_side // 65536)
    big = [np.ascontiguousarray(f[k], np.float32).ravel()
           for k in ("mean_u", "var_u", "mean_v", "var_v")]
    del f

    def planes(side):
        return [x[: side * side].reshape(side, side) for x in big]

    sides = [4096, 2353, 776, 256]
    srv = P.Server(hbm_budget=24 << 30, n_streams=2)
    srv.reserve_staging(big_side ** 2, 6)
    puts = [srv.put_field(fid, *planes(s)) for fid, s in enumerate(sides)]
    rng = np.random.default_rng(11)
    reqs = []
    for r in range(24):
        fid = r % len(sides)
        k = int(rng.integers(1, 5))
        iso = ((rng.random(k) - 0.5) * 0.05).astype(np.float32)
        s = sides[fid]
        out = torch.empty((k, s - 1, s - 1), device="cuda")
        reqs.append((fid, iso, out, srv.submit_lcp(fid, iso, out)))
    for t in puts:
        assert srv.wait(t) == 0
    for _, _, _, t in reqs:
        assert srv.wait(t) == 0
    torch.cuda.synchronize()
    worst = 0.0
    stored = {}
    for fid, iso, out, _ in reqs:
        s = sides[fid]
        if fid not in stored:
            stored[fid] = [p.astype(np.float64) for p in planes(s)]
        mom = stored[fid]
        bands = [(0, s - 1)] if s <= 776 else [(0, 2), (s // 2, s // 2 + 2), (s - 3, s - 1)]
        for j0, j1 in bands:
            ref = oracle_rows(mom, 1.0, 1.0, iso, j0, j1)
            worst = max(worst, float(np.max(np.abs(host64(out[:, j0:j1, :]) - ref))))
    st = srv.stats()
    print(f"\n[c5 served] max |LCP - oracle| = {worst:.3e}; launches {st['launches']}, "
          f"peak {st['peak_bytes'] / 2**30:.2f} GiB")
    assert worst <= LCP_TOL
    assert st["failed"] == 0 and st["peak_bytes"] <= 24 << 30
    srv.close()
