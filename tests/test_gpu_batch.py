"""Batched persistent launch: bitwise equal to per-field launches (same tile
code), correct against the oracle, and stable under graph replay with
isovalue updates between replays."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2510_01190_amd as P
import synth
from gpu_util import TORCH_DT, host64

pytestmark = pytest.mark.gpu


def _fields(n, lo, hi, seed, dt="f32", kmax=16):
    rng = np.random.default_rng(seed)
    sizes = synth.batch_sizes(n, lo, hi, seed)
    sizes[0] = (2, 2)
    sizes[1] = (2, 37)
    sizes[2] = (129, 2)
    out = []
    for k, (ny, nx) in enumerate(sizes):
        f = synth.gen_moments(ny, nx, seed * 1000 + k, n_features=max(1, ny * nx // 3000))
        K = int(rng.integers(1, kmax + 1))
        iso = rng.uniform(-0.1, 0.1, K).astype(np.float32)
        d = {key: torch.from_numpy(f[key]).to(TORCH_DT[dt]).cuda()
             for key in ("mean_u", "var_u", "mean_v", "var_v")}
        d.update(isovalues=torch.from_numpy(iso).cuda(), dx=1.0 + 0.5 * (k % 3), dy=1.0,
                 iso_host=iso)
        out.append(d)
    return out


def _per_field(f):
    return P.lcp_from_moments(f["mean_u"], f["var_u"], f["mean_v"], f["var_v"],
                              f["iso_host"], dx=f["dx"], dy=f["dy"])


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_per_field_launches(graph):
    fields = _fields(40, 2, 300, seed=1)
    b = P.Batch(fields, graph=graph)
    b.launch()
    torch.cuda.synchronize()
    for f, g in zip(fields, b.fields):
        assert torch.equal(g["lcp"], _per_field(f))
    b.close()


def test_batch_against_oracle():
    fields = _fields(12, 2, 200, seed=2)
    b = P.Batch(fields, graph=False)
    b.launch()
    torch.cuda.synchronize()
    for f, g in zip(fields, b.fields):
        mom = [host64(f[k]) for k in ("mean_u", "var_u", "mean_v", "var_v")]
        ref = O.lcp(*O.divergence_gaussian(*mom, f["dx"], f["dy"]), f["iso_host"])
        assert np.max(np.abs(host64(g["lcp"]) - ref)) <= 1e-5
    b.close()


def test_graph_replays_with_isovalue_updates():
    fields = _fields(20, 16, 400, seed=3, kmax=4)
    b = P.Batch(fields, graph=True)
    rng = np.random.default_rng(9)
    for replay in range(4):
        for f in fields:  # move every slider: device-side update, then eager work
            new = rng.uniform(-0.1, 0.1, f["isovalues"].numel()).astype(np.float32)
            f["isovalues"].copy_(torch.from_numpy(new))
            f["iso_host"] = new
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for f, g in zip(fields, b.fields):
            assert torch.equal(g["lcp"], _per_field(f)), f"replay {replay}"
        torch.cuda.synchronize()
    b.close()


def test_autotuned_batch(tmp_path, monkeypatch):
    monkeypatch.setenv("PDIV_TUNE_CACHE", str(tmp_path / "tune.json"))
    fields = _fields(30, 32, 600, seed=4, kmax=4)
    b = P.Batch(fields, graph=True, autotune=True)
    info = b.info()
    assert info["band_rows"] in (8, 16, 32, 64) and info["n_tiles"] > 0
    b.launch()
    torch.cuda.synchronize()
    for f, g in zip(fields, b.fields):
        assert torch.equal(g["lcp"], _per_field(f))
    b.close()


@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_batch_16bit_storage(dt):
    fields = _fields(10, 2, 150, seed=5, dt=dt)
    b = P.Batch(fields, graph=False)
    b.launch()
    torch.cuda.synchronize()
    for f, g in zip(fields, b.fields):
        assert torch.equal(g["lcp"], _per_field(f))
    b.close()


def test_batch_pitched_outputs():
    """Fields whose outputs have padded rows: same maps as the dense per-field
    launches, padding untouched."""
    fields = _fields(10, 2, 300, seed=6)
    bufs = []
    for k, f in enumerate(fields):
        ny, nx = f["mean_u"].shape
        K = f["iso_host"].size
        pitch = (nx - 1 + 31) // 32 * 32 + 32 * (k % 2)
        if k % 3 == 2:  # maps interleaved by rows
            buf = torch.full((ny - 1, K, pitch), -3.0, device="cuda")
            f["lcp"] = buf.permute(1, 0, 2)[:, :, : nx - 1]
        else:
            buf = torch.full((K, ny - 1, pitch), -3.0, device="cuda")
            f["lcp"] = buf[:, :, : nx - 1]
        bufs.append((buf, nx))
    b = P.Batch(fields, graph=True)
    b.launch()
    torch.cuda.synchronize()
    for f, g, (buf, nx) in zip(fields, b.fields, bufs):
        assert torch.equal(g["lcp"], _per_field(f))
        assert bool((buf[..., nx - 1:] == -3.0).all())
    b.close()


def test_autotuned_batch_with_line_aligned_outputs(tmp_path, monkeypatch):
    """With every output row on a 128-byte line the autotuner also times the
    paired tile layout; whichever it keeps, the maps are the per-field ones,
    and a second batch reads the choice back from the cache file."""
    monkeypatch.setenv("PDIV_TUNE_CACHE", str(tmp_path / "tune.json"))
    fields = _fields(24, 40, 400, seed=9, kmax=16)
    for f in fields:
        ny, nx = f["mean_u"].shape
        f["lcp"] = P.empty_lcp(f["iso_host"].size, ny, nx)
    b = P.Batch(fields, graph=True, autotune=True)
    b.launch()
    torch.cuda.synchronize()
    info = b.info()
    assert info["strip_cells"] in (126, 128)
    for f, g in zip(fields, b.fields):
        assert torch.equal(g["lcp"], _per_field(f))
    b.close()
    assert "/l1/" in (tmp_path / "tune.json").read_text()
    b2 = P.Batch(fields, graph=False, autotune=True)
    assert b2.info() == info
    b2.close()
