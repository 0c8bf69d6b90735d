"""pdiv_spaghetti_noalloc (the entry point that allocates nothing, its
workspace a static device array) against pdiv_spaghetti with a caller
workspace: offsets and segments bit for bit, on two calls in a row, the
second with a smaller input, so that what the first call left in the shared
workspace cannot leak into the second's result."""

import ctypes

import numpy as np
import pytest
import torch

import paper_2510_01190_amd as P
import synth
from gpu_util import TORCH_DT

pytestmark = pytest.mark.gpu

_v = ctypes.c_void_p


def _members(m, ny, nx, seed, dt):
    e = synth.gen_ensemble(ny, nx, m, seed=seed, n_features=3, dtype=np.float32)
    return [torch.from_numpy(e[k]).to(TORCH_DT[dt]).cuda() for k in ("u_members", "v_members")]


def _run(noalloc, u, v, c, dx, dy):
    """Count pass (max_segments 0), then the write pass, through the C ABI."""
    L = P.lib()
    m, ny, nx = u.shape
    code = {"torch.float32": 0, "torch.float16": 1, "torch.bfloat16": 2}[str(u.dtype)]
    offs = torch.empty(m * (ny - 1) + 1, dtype=torch.int64, device="cuda")
    stream = _v(torch.cuda.current_stream().cuda_stream)
    work = None if noalloc else torch.empty((m, ny, nx), dtype=torch.float32, device="cuda")

    def call(segs, cap):
        sp = _v(segs.data_ptr()) if segs is not None else None
        if noalloc:
            return L.pdiv_spaghetti_noalloc(_v(u.data_ptr()), _v(v.data_ptr()), code, m, ny, nx,
                                            0, dx, dy, ctypes.c_float(c), _v(offs.data_ptr()),
                                            sp, cap, stream)
        return L.pdiv_spaghetti(_v(u.data_ptr()), _v(v.data_ptr()), code, m, ny, nx, 0, dx, dy,
                                ctypes.c_float(c), _v(work.data_ptr()), _v(offs.data_ptr()), sp,
                                cap, stream)

    assert call(None, 0) == 0, L.pdiv_last_error()
    n = int(offs[-1].item())
    segs = torch.full((max(n, 1), 4), -7.0, device="cuda")
    assert call(segs, n) == 0, L.pdiv_last_error()
    torch.cuda.synchronize()
    return offs.cpu(), segs[:n].cpu()


def test_noalloc_equals_workspace_call_on_two_calls_in_a_row():
    cases = [(12, 300, 257, 0.01, "f32", (1.0, 1.0)),   # 0.9 M floats of workspace
             (3, 40, 70, -0.02, "bf16", (0.5, 2.0))]    # smaller: stale data beyond it
    for m, ny, nx, c, dt, (dx, dy) in cases:
        u, v = _members(m, ny, nx, seed=m + ny, dt=dt)
        o1, s1 = _run(True, u, v, c, dx, dy)
        o0, s0 = _run(False, u, v, c, dx, dy)
        assert torch.equal(o1, o0)
        assert s1.shape[0] > 0 and torch.equal(s1, s0)


def test_noalloc_rejects_a_workspace_beyond_its_limit():
    L = P.lib()
    fake = _v(0x1000)  # never dereferenced: the size check comes first
    offs = _v(0x2000)
    st = L.pdiv_spaghetti_noalloc(fake, fake, 0, 17, 1024, 1024, 0, 1.0, 1.0,
                                  ctypes.c_float(0.0), offs, None, 0, None)
    assert st == 1 and "workspace" in L.pdiv_last_error().decode()
