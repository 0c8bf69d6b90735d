"""GPU parity of the isocontour geometry (marching squares: the mean-field
contour and the spaghetti plot of Section 4) against the oracle, through the
C ABI.  The case decisions compare float32 values on both sides (and the
saddle centre is evaluated in float32 by both), so the segment lists match
one to one; the points differ only by the float32 evaluation of
t = (c - p) / (q - p) and i + t: at most 4 u (1 + |x|)."""

import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import paper_2510_01190_amd as P
import synth
from gpu_util import U32, host64

pytestmark = pytest.mark.gpu


def _compare(field32, c):
    g = host64(P.isocontour(torch.from_numpy(field32).cuda(), c))
    r = O.marching_squares(field32.astype(np.float64), float(np.float32(c)))
    assert g.shape == r.shape, (g.shape, r.shape)
    assert np.all(np.abs(g - r) <= 4 * U32 * (1 + np.abs(r)))
    return r


def _fields():
    rng = np.random.default_rng(6)
    y, x = np.mgrid[0:45, 0:67].astype(np.float64)
    yield "plane", (0.3 * x - 0.8 * y).astype(np.float32), [-3.0, 0.0, 7.5]
    yield "circle", ((x - 30.2) ** 2 + (y - 20.7) ** 2).astype(np.float32), [100.0, 300.5]
    yield "ties", np.round(rng.normal(0, 1, (33, 130)), 1).astype(np.float32), [0.0, 0.3, -1.0]
    yield "noise", rng.normal(0, 1, (130, 65)).astype(np.float32), [0.05]
    yield "saddles", np.tile(np.array([[1, 0], [0, 1]], np.float32), (20, 40)), [0.5, 0.25]
    yield "tiny", np.array([[0.0, 1.0], [1.0, 0.0]], np.float32), [0.5]
    yield "wide", rng.normal(0, 1, (3, 300)).astype(np.float32), [0.0, 1.5]


@pytest.mark.parametrize("name,field,isos", list(_fields()), ids=[f[0] for f in _fields()])
def test_matches_oracle(name, field, isos):
    for c in isos:
        _compare(field, c)


def test_offsets_and_a_short_buffer():
    rng = np.random.default_rng(1)
    f = rng.normal(0, 1, (40, 150)).astype(np.float32)
    ft = torch.from_numpy(f).cuda()
    r = O.marching_squares(f.astype(np.float64), 0.2)
    offs = torch.empty(40, dtype=torch.int64, device="cuda")
    cap = len(r) // 2
    segs = torch.full((len(r), 4), -7.0, device="cuda")
    L = P.lib()
    st = L.pdiv_isocontour(ctypes.c_void_p(ft.data_ptr()), 40, 150, ctypes.c_float(0.2),
                           ctypes.c_void_p(offs.data_ptr()), ctypes.c_void_p(segs.data_ptr()), cap,
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    o = offs.cpu().numpy()
    assert o[-1] == len(r) and o[0] == 0 and np.all(np.diff(o) >= 0)
    # the segments of cell row j start at offs[j] and lie in that row
    for j in range(39):
        lo, hi = o[j], o[j + 1]
        rows = np.minimum(r[lo:hi, 1], r[lo:hi, 3])
        assert np.all((rows >= j) & (rows <= j + 1))
    g = host64(segs)
    assert np.all(np.abs(g[:cap] - r[:cap]) <= 4 * U32 * (1 + np.abs(r[:cap])))
    assert np.all(g[cap:] == -7.0)  # past max_segments nothing is written


def test_mean_field_contour_of_the_ensemble():
    """The mean-field isocontour of the fitted 721 x 1440 ensemble's
    divergence at its isovalues: the oracle's fit, stored as float32, and its
    float32 divergence are the field both sides contour."""
    e = synth.config_c2()
    mom32 = [m.astype(np.float32) for m in O.moments(e["u_members"], e["v_members"], 1)]
    d32 = O.divergence_gaussian_f32(*mom32, 1.0, 1.0)[0]
    for c in e["isovalues"][[0, 4, 7]]:
        r = _compare(d32, c)
        assert len(r) > 100


def test_spaghetti_matches_per_member_contours():
    e = synth.gen_ensemble(60, 90, 6, seed=4, n_features=3, dtype=np.float32)
    u = torch.from_numpy(e["u_members"]).cuda()
    v = torch.from_numpy(e["v_members"]).cuda()
    sp = P.spaghetti(u, v, 0.02)
    assert len(sp) == 6
    zero = torch.zeros((60, 90), device="cuda")
    z64 = np.zeros((60, 90))
    for m in range(6):
        d, _ = P.divergence_gaussian(u[m].contiguous(), zero, v[m].contiguous(), zero)
        # the member's divergence is Eq. 1 in float32, as the oracle rounds it
        um, vm = e["u_members"][m].astype(np.float64), e["v_members"][m].astype(np.float64)
        d32 = O.divergence_gaussian_f32(um, z64, vm, z64, 1.0, 1.0)[0]
        assert np.array_equal(d.cpu().numpy(), d32)
        ref_d = O.fd_divergence(um, vm, 1.0, 1.0)
        scale = max(np.abs(um).max(), np.abs(vm).max())
        assert np.max(np.abs(d32 - ref_d)) <= 8 * U32 * scale
        r = O.marching_squares(d32.astype(np.float64), float(np.float32(0.02)))
        g = host64(sp[m])
        assert g.shape == r.shape
        assert np.all(np.abs(g - r) <= 4 * U32 * (1 + np.abs(r)))
        # one batched call gives bitwise the per-member contours
        assert torch.equal(sp[m], P.isocontour(d, 0.02))


@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_spaghetti_16bit_members_and_spacing(dt):
    from gpu_util import TORCH_DT
    e = synth.gen_ensemble(33, 130, 4, seed=8, n_features=2, dtype=np.float32)
    u = torch.from_numpy(e["u_members"]).to(TORCH_DT[dt]).cuda()
    v = torch.from_numpy(e["v_members"]).to(TORCH_DT[dt]).cuda()
    sp = P.spaghetti(u, v, -0.01, dx=0.5, dy=2.0)
    zero = torch.zeros((33, 130), dtype=TORCH_DT[dt], device="cuda")
    for m in range(4):
        d, _ = P.divergence_gaussian(u[m].contiguous(), zero, v[m].contiguous(), zero, 0.5, 2.0)
        assert torch.equal(sp[m], P.isocontour(d, -0.01))
