"""Python binding of libpdiv, the gfx950 probabilistic local-divergence library.

Thin ctypes layer over the C ABI declared in include/pdiv.h: it checks tensor
shapes, passes device pointers and the current HIP stream, and raises
PdivError on a non-OK status.  All computation happens in the library's HIP
kernels; there is no fallback of any kind.  If libpdiv.so has not been built
(python -m paper_2510_01190_amd.build_lib), every call raises.

Tensors are torch CUDA tensors (ROCm): torch provides device memory and
streams only.  Planes are row-major [ny][nx] with x fastest; LCP outputs are
[n_iso][ny-1][nx-1] float32.
"""

from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

__all__ = [
    "PdivError", "lib", "moments", "divergence_gaussian", "lcp", "lcp_from_moments",
    "mc_lcp", "mc_sample_field", "empty_lcp", "Batch", "Server", "STATUS", "MAX_ISO",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdiv.so")
MAX_ISO = 256

STATUS = {0: "PDIV_OK", 1: "PDIV_ERR_INVALID", 2: "PDIV_ERR_UNSUPPORTED", 3: "PDIV_ERR_NOMEM",
          4: "PDIV_ERR_DEVICE", 5: "PDIV_ERR_BUSY", 6: "PDIV_ERR_TIMEOUT"}
_DT = {"float32": 0, "float16": 1, "bfloat16": 2}
_TIMEOUT = 6  # PDIV_ERR_TIMEOUT

_c = ctypes
_p = _c.c_void_p
_i64 = _c.c_int64
_i32 = _c.c_int32
_f64 = _c.c_double
_u64 = _c.c_uint64
_fp = _c.POINTER(_c.c_float)


class PdivError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class _Field(_c.Structure):
    _fields_ = [("mean_u", _p), ("var_u", _p), ("mean_v", _p), ("var_v", _p),
                ("ny", _i64), ("nx", _i64), ("dx", _f64), ("dy", _f64),
                ("isovalues", _p), ("n_iso", _i32), ("lcp", _p), ("lcp_row_pitch", _i64),
                ("lcp_plane_stride", _i64)]


class ServerStats(_c.Structure):
    _fields_ = [("done", _u64), ("failed", _u64), ("launches", _u64),
                ("p50_us", _f64), ("p99_us", _f64), ("p50_new_us", _f64), ("p99_new_us", _f64),
                ("p50_slider_us", _f64), ("p99_slider_us", _f64), ("lcp_cells", _f64),
                ("resident_bytes", _c.c_size_t), ("peak_bytes", _c.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_SIGS = {
    "pdiv_moments": [_p, _p, _c.c_int, _i64, _i64, _i64, _i64, _i32, _p, _p, _p, _p, _c.c_int, _p],
    "pdiv_divergence_gaussian": [_p, _p, _p, _p, _c.c_int, _i64, _i64, _f64, _f64, _p, _p, _p],
    "pdiv_lcp": [_p, _p, _i64, _i64, _fp, _i32, _p, _i64, _i64, _p],
    "pdiv_speed_gradient_moments": [_p, _p, _c.c_int, _i64, _i64, _i64, _i64, _f64, _f64, _i32,
                                    _p, _p, _p, _p, _c.c_int, _p],
    "pdiv_isocontour": [_p, _i64, _i64, _c.c_float, _p, _p, _i64, _p],
    "pdiv_spaghetti": [_p, _p, _c.c_int, _i64, _i64, _i64, _i64, _f64, _f64, _c.c_float, _p, _p,
                       _p, _i64, _p],
    "pdiv_spaghetti_noalloc": [_p, _p, _c.c_int, _i64, _i64, _i64, _i64, _f64, _f64,
                               _c.c_float, _p, _p, _i64, _p],
    "pdiv_divergence_gaussian_3d": [_p, _p, _p, _p, _p, _p, _c.c_int, _i64, _i64, _i64, _f64,
                                    _f64, _f64, _p, _p, _p],
    "pdiv_lcp_3d": [_p, _p, _i64, _i64, _i64, _fp, _i32, _p, _i64, _i64, _p],
    "pdiv_lcp_3d_from_moments": [_p, _p, _p, _p, _p, _p, _c.c_int, _i64, _i64, _i64, _f64, _f64,
                                 _f64, _fp, _i32, _p, _i64, _i64, _p],
    "pdiv_mc_lcp": [_p, _p, _p, _p, _c.c_int, _i64, _i64, _f64, _f64, _fp, _i32, _i64, _u64,
                    _c.c_uint32, _p, _p],
    "pdiv_lcp_from_moments": [_p, _p, _p, _p, _c.c_int, _i64, _i64, _f64, _f64, _fp, _i32, _p,
                              _i64, _i64, _p],
    "pdiv_mc_sample_field": [_p, _p, _p, _p, _c.c_int, _i64, _i64, _i64, _u64, _p, _p, _p],
    "pdiv_batch_create": [_c.POINTER(_Field), _i32, _c.c_int, _c.c_uint32, _p, _c.POINTER(_p)],
    "pdiv_batch_launch": [_p, _p],
    "pdiv_batch_info": [_p, _c.POINTER(_i32), _c.POINTER(_i32), _c.POINTER(_i64)],
    "pdiv_batch_destroy": [_p],
    "pdiv_server_create": [_c.c_size_t, _i32, _c.POINTER(_p)],
    "pdiv_server_put_field": [_p, _u64, _p, _p, _p, _p, _c.c_int, _i64, _i64, _f64, _f64,
                              _c.POINTER(_u64)],
    "pdiv_server_reserve_staging": [_p, _i64, _c.c_int, _i32],
    "pdiv_server_submit_lcp": [_p, _u64, _fp, _i32, _p, _c.POINTER(_u64)],
    "pdiv_server_wait": [_p, _u64, _i64, _c.POINTER(_c.c_int)],
    "pdiv_server_stats": [_p, _c.POINTER(ServerStats)],
    "pdiv_server_destroy": [_p],
    "pdiv_set_lcp_band_rows": [_i32],
    "pdiv_set_debug": [_c.c_uint32],
}
EXPORTS = list(_SIGS) + ["pdiv_status_string", "pdiv_last_error", "pdiv_version"]

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libpdiv.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"libpdiv.so not found at {LIB_PATH}; build it with "
                "`python -m paper_2510_01190_amd.build_lib` (there is no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _c.c_int
        for name in ("pdiv_status_string",):
            getattr(L, name).argtypes = [_c.c_int]
            getattr(L, name).restype = _c.c_char_p
        for name in ("pdiv_last_error", "pdiv_version"):
            getattr(L, name).argtypes = []
            getattr(L, name).restype = _c.c_char_p
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise PdivError(status, lib().pdiv_last_error().decode())


def _torch():
    import torch
    return torch


def _stream():
    return _p(_torch().cuda.current_stream().cuda_stream)


def _dtype_code(t) -> int:
    name = str(t.dtype).replace("torch.", "")
    if name not in _DT:
        raise TypeError(f"unsupported dtype {t.dtype}; use float32, float16 or bfloat16")
    return _DT[name]


def _dev(t, name, shape=None, dtype=None):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    return _p(t.data_ptr())


def _lcp_out(t, k, ny, nx):
    """Pointer, row pitch and plane stride (floats) of an LCP output: a
    [k][ny-1][nx-1] float32 device tensor whose cells are contiguous within a
    row -- dense, or a strided view such as empty_lcp returns.  The library
    checks that the maps do not overlap."""
    if not t.is_cuda:
        raise ValueError("out must be a device tensor")
    if t.dtype != _torch().float32:
        raise ValueError(f"out has dtype {t.dtype}, expected torch.float32")
    if tuple(t.shape) != (k, ny - 1, nx - 1):
        raise ValueError(f"out has shape {tuple(t.shape)}, expected {(k, ny - 1, nx - 1)}")
    s0, s1, s2 = t.stride()
    if s2 != 1 and nx > 2:
        raise ValueError("out: the cells of a row must be contiguous")
    # a single row or map: its stride is free in torch; keep it if it is one
    pitch = s1 if (ny > 2 or s1 >= nx - 1) else nx - 1
    plane = s0 if k > 1 else 0
    if pitch < nx - 1 or (k > 1 and plane < 1):
        raise ValueError("out: rows or maps overlap")
    return _p(t.data_ptr()), pitch, plane


def empty_lcp(k: int, ny: int, nx: int, pitch: int = None, interleave_rows: bool = False,
              device="cuda"):
    """Uninitialised LCP output [k][ny-1][nx-1] whose rows are `pitch` floats
    long (default: nx-1 rounded up to a multiple of 32 floats, so that every
    row starts on a 128-byte line); padding floats are never written.
    interleave_rows: the k maps' rows j are adjacent in memory (a
    [ny-1][k][pitch] buffer viewed as [k][ny-1][nx-1]), the layout the
    kernels write fastest on gfx950."""
    torch = _torch()
    if pitch is None:
        pitch = (nx - 1 + 31) // 32 * 32
    if pitch < nx - 1:
        raise ValueError("pitch must be >= nx - 1")
    if interleave_rows:
        buf = torch.empty((ny - 1, k, pitch), dtype=torch.float32, device=device)
        return buf.permute(1, 0, 2)[:, :, : nx - 1]
    buf = torch.empty((k, ny - 1, pitch), dtype=torch.float32, device=device)
    return buf[:, :, : nx - 1]


def _lcp3_out(t, k, nz, ny, nx):
    """Pointer, row pitch and map stride (floats) of a 3D LCP output: a
    [k][nz-1][ny-1][nx-1] float32 device tensor whose cells are contiguous
    within a row and whose layers are (ny-1) rows apart -- dense, or a view
    such as empty_lcp_3d returns."""
    if not t.is_cuda:
        raise ValueError("out must be a device tensor")
    if t.dtype != _torch().float32:
        raise ValueError(f"out has dtype {t.dtype}, expected torch.float32")
    shape = (k, nz - 1, ny - 1, nx - 1)
    if tuple(t.shape) != shape:
        raise ValueError(f"out has shape {tuple(t.shape)}, expected {shape}")
    s0, s1, s2, s3 = t.stride()
    if s3 != 1 and nx > 2:
        raise ValueError("out: the cells of a row must be contiguous")
    pitch = s2 if ny > 2 else (s1 if nz > 2 else max(s2, nx - 1))
    if pitch < nx - 1:
        raise ValueError("out: rows overlap")
    if nz > 2 and s1 != (ny - 1) * pitch:
        raise ValueError("out: layers must follow each other, (ny-1) rows apart")
    plane = s0 if k > 1 else 0
    return _p(t.data_ptr()), pitch, plane


def empty_lcp_3d(k: int, nz: int, ny: int, nx: int, pitch: int = None, device="cuda"):
    """Uninitialised 3D LCP output [k][nz-1][ny-1][nx-1] whose rows are
    `pitch` floats long (default: nx-1 rounded up to a multiple of 32 floats,
    so that every row starts on a 128-byte line, the layout the kernels write
    fastest); padding floats are never written."""
    torch = _torch()
    if pitch is None:
        pitch = (nx - 1 + 31) // 32 * 32
    if pitch < nx - 1:
        raise ValueError("pitch must be >= nx - 1")
    buf = torch.empty((k, nz - 1, ny - 1, pitch), dtype=torch.float32, device=device)
    return buf[..., : nx - 1]


def _iso_arr(isovalues):
    iso = np.ascontiguousarray(np.atleast_1d(np.asarray(isovalues, np.float32)))
    return iso, iso.ctypes.data_as(_fp)


def _moment_ptrs(mean_u, var_u, mean_v, var_v):
    ny, nx = mean_u.shape
    dt = mean_u.dtype
    ptrs = [_dev(t, n, (ny, nx), dt) for t, n in
            ((mean_u, "mean_u"), (var_u, "var_u"), (mean_v, "mean_v"), (var_v, "var_v"))]
    return ptrs, ny, nx, _dtype_code(mean_u)


def set_lcp_band_rows(rows: int):
    """Cell rows per wave band of the closed-form LCP kernels (0 = built-in choice)."""
    _check(lib().pdiv_set_lcp_band_rows(rows))


DEBUG_POISON_LDS, DEBUG_CHECK_INPUTS, DEBUG_LOG = 1, 2, 4


def set_debug(flags: int):
    """Process-wide checking modes, an OR of DEBUG_* (0 switches all off)."""
    _check(lib().pdiv_set_debug(flags))


def moments(u_members, v_members, ddof: int = 1, out_dtype=None):
    """Per-point mean and variance over members: inputs [M][ny][nx] -> 4 planes [ny][nx]."""
    torch = _torch()
    m, ny, nx = u_members.shape
    od = out_dtype or torch.float32
    outs = [torch.empty((ny, nx), dtype=od, device=u_members.device) for _ in range(4)]
    pu = _dev(u_members, "u_members", (m, ny, nx))
    pv = _dev(v_members, "v_members", (m, ny, nx), u_members.dtype)
    _check(lib().pdiv_moments(pu, pv, _dtype_code(u_members), m, ny, nx, 0, ddof,
                              *[_p(o.data_ptr()) for o in outs], _dtype_code(outs[0]), _stream()))
    return tuple(outs)


def speed_gradient_moments(u_members, v_members, dx: float = 1.0, dy: float = 1.0,
                           ddof: int = 1, out_dtype=None):
    """The Red Sea pre-stage: per member the gradient of the speed, fitted
    over members -> (mean_gx, var_gx, mean_gy, var_gy) planes [ny][nx], ready
    for lcp_from_moments."""
    torch = _torch()
    m, ny, nx = u_members.shape
    od = out_dtype or torch.float32
    outs = [torch.empty((ny, nx), dtype=od, device=u_members.device) for _ in range(4)]
    pu = _dev(u_members, "u_members", (m, ny, nx))
    pv = _dev(v_members, "v_members", (m, ny, nx), u_members.dtype)
    _check(lib().pdiv_speed_gradient_moments(pu, pv, _dtype_code(u_members), m, ny, nx, 0, dx,
                                             dy, ddof, *[_p(o.data_ptr()) for o in outs],
                                             _dtype_code(outs[0]), _stream()))
    return tuple(outs)


def divergence_gaussian(mean_u, var_u, mean_v, var_v, dx: float = 1.0, dy: float = 1.0):
    """Eq. 2-3: (div_mean, div_var) float32 planes."""
    torch = _torch()
    ptrs, ny, nx, dt = _moment_ptrs(mean_u, var_u, mean_v, var_v)
    dm = torch.empty((ny, nx), dtype=torch.float32, device=mean_u.device)
    dv = torch.empty_like(dm)
    _check(lib().pdiv_divergence_gaussian(*ptrs, dt, ny, nx, dx, dy, _p(dm.data_ptr()),
                                          _p(dv.data_ptr()), _stream()))
    return dm, dv


def lcp(div_mean, div_var, isovalues, out=None):
    """Closed-form LCP [K][ny-1][nx-1] from divergence Gaussians; `out` may be
    dense or a row-padded view (empty_lcp)."""
    torch = _torch()
    ny, nx = div_mean.shape
    pm = _dev(div_mean, "div_mean", (ny, nx), torch.float32)
    pv = _dev(div_var, "div_var", (ny, nx), torch.float32)
    iso, ip = _iso_arr(isovalues)
    if out is None:
        out = torch.empty((iso.size, ny - 1, nx - 1), dtype=torch.float32, device=div_mean.device)
    po, pitch, plane = _lcp_out(out, iso.size, ny, nx)
    _check(lib().pdiv_lcp(pm, pv, ny, nx, ip, iso.size, po, pitch, plane, _stream()))
    return out


def isocontour(field, isovalue):
    """Marching-squares segments [n][4] (x0, y0, x1, y1) of a [ny][nx]
    float32 field at isovalue, cell by cell in row-major order."""
    torch = _torch()
    ny, nx = field.shape
    pf = _dev(field, "field", (ny, nx), torch.float32)
    offs = torch.empty(ny, dtype=torch.int64, device=field.device)
    c = float(np.float32(isovalue))
    _check(lib().pdiv_isocontour(pf, ny, nx, c, _p(offs.data_ptr()), None, 0, _stream()))
    n = int(offs[ny - 1].item())
    segs = torch.empty((n, 4), dtype=torch.float32, device=field.device)
    if n:
        _check(lib().pdiv_isocontour(pf, ny, nx, c, _p(offs.data_ptr()), _p(segs.data_ptr()), n,
                                     _stream()))
    return segs


def spaghetti(u_members, v_members, isovalue, dx: float = 1.0, dy: float = 1.0):
    """Per-member isocontours of the divergence (Eq. 1, each member taken as a
    deterministic field) at isovalue, in one library call: a list of [n_m][4]
    segment tensors (views of one buffer)."""
    torch = _torch()
    m, ny, nx = u_members.shape
    pu = _dev(u_members, "u_members", (m, ny, nx))
    pv = _dev(v_members, "v_members", (m, ny, nx), u_members.dtype)
    work = torch.empty((m, ny, nx), dtype=torch.float32, device=u_members.device)
    offs = torch.empty(m * (ny - 1) + 1, dtype=torch.int64, device=u_members.device)
    c = float(np.float32(isovalue))
    args = (pu, pv, _dtype_code(u_members), m, ny, nx, 0, dx, dy, c, _p(work.data_ptr()),
            _p(offs.data_ptr()))
    _check(lib().pdiv_spaghetti(*args, None, 0, _stream()))
    n = int(offs[-1].item())
    segs = torch.empty((max(n, 1), 4), dtype=torch.float32, device=u_members.device)
    _check(lib().pdiv_spaghetti(*args, _p(segs.data_ptr()), n, _stream()))
    bounds = offs[::ny - 1].cpu().tolist()
    return [segs[bounds[q]:bounds[q + 1]] for q in range(m)]


def divergence_gaussian_3d(mean_u, var_u, mean_v, var_v, mean_w, var_w, dx: float = 1.0,
                           dy: float = 1.0, dz: float = 1.0):
    """Eq. 2-3 with the z term for a 3D field (six [nz][ny][nx] planes of one
    dtype): (div_mean, div_var) float32 [nz][ny][nx]."""
    torch = _torch()
    nz, ny, nx = mean_u.shape
    dt = mean_u.dtype
    ptrs = [_dev(t, n, (nz, ny, nx), dt) for t, n in
            ((mean_u, "mean_u"), (var_u, "var_u"), (mean_v, "mean_v"), (var_v, "var_v"),
             (mean_w, "mean_w"), (var_w, "var_w"))]
    dm = torch.empty((nz, ny, nx), dtype=torch.float32, device=mean_u.device)
    dv = torch.empty_like(dm)
    _check(lib().pdiv_divergence_gaussian_3d(*ptrs, _dtype_code(mean_u), nz, ny, nx, dx, dy, dz,
                                             _p(dm.data_ptr()), _p(dv.data_ptr()), _stream()))
    return dm, dv


def lcp_3d_from_moments(mean_u, var_u, mean_v, var_v, mean_w, var_w, isovalues,
                        dx: float = 1.0, dy: float = 1.0, dz: float = 1.0, out=None):
    """Fused 3D Eq. 2-3 + 8-corner LCP [K][nz-1][ny-1][nx-1] from the six
    [nz][ny][nx] moment volumes; `out` may be dense or a row-padded view
    (empty_lcp_3d)."""
    torch = _torch()
    nz, ny, nx = mean_u.shape
    dt = mean_u.dtype
    ptrs = [_dev(t, n, (nz, ny, nx), dt) for t, n in
            ((mean_u, "mean_u"), (var_u, "var_u"), (mean_v, "mean_v"), (var_v, "var_v"),
             (mean_w, "mean_w"), (var_w, "var_w"))]
    iso, ip = _iso_arr(isovalues)
    if out is None:
        out = torch.empty((iso.size, nz - 1, ny - 1, nx - 1), dtype=torch.float32,
                          device=mean_u.device)
    po, pitch, plane = _lcp3_out(out, iso.size, nz, ny, nx)
    _check(lib().pdiv_lcp_3d_from_moments(*ptrs, _dtype_code(mean_u), nz, ny, nx, dx, dy, dz, ip,
                                          iso.size, po, pitch, plane, _stream()))
    return out


def lcp_3d(div_mean, div_var, isovalues, out=None):
    """8-corner LCP [K][nz-1][ny-1][nx-1] from 3D divergence Gaussians; `out`
    may be dense or a row-padded view (empty_lcp_3d)."""
    torch = _torch()
    nz, ny, nx = div_mean.shape
    pm = _dev(div_mean, "div_mean", (nz, ny, nx), torch.float32)
    pv = _dev(div_var, "div_var", (nz, ny, nx), torch.float32)
    iso, ip = _iso_arr(isovalues)
    if out is None:
        out = torch.empty((iso.size, nz - 1, ny - 1, nx - 1), dtype=torch.float32,
                          device=div_mean.device)
    po, pitch, plane = _lcp3_out(out, iso.size, nz, ny, nx)
    _check(lib().pdiv_lcp_3d(pm, pv, nz, ny, nx, ip, iso.size, po, pitch, plane, _stream()))
    return out


def lcp_from_moments(mean_u, var_u, mean_v, var_v, isovalues, dx: float = 1.0,
                     dy: float = 1.0, out=None):
    """Fused Eq. 2-3 + closed-form LCP [K][ny-1][nx-1]; `out` may be dense or a
    row-padded view (empty_lcp)."""
    torch = _torch()
    ptrs, ny, nx, dt = _moment_ptrs(mean_u, var_u, mean_v, var_v)
    iso, ip = _iso_arr(isovalues)
    if out is None:
        out = torch.empty((iso.size, ny - 1, nx - 1), dtype=torch.float32, device=mean_u.device)
    po, pitch, plane = _lcp_out(out, iso.size, ny, nx)
    _check(lib().pdiv_lcp_from_moments(*ptrs, dt, ny, nx, dx, dy, ip, iso.size, po, pitch,
                                       plane, _stream()))
    return out


MC_MODES = {"vector": 0, "vertex": 1}


def mc_lcp(mean_u, var_u, mean_v, var_v, isovalues, n_samples: int, seed: int,
           dx: float = 1.0, dy: float = 1.0, out=None, mode: str = "vector"):
    """Monte Carlo LCP [K][ny-1][nx-1]: mode "vector" samples the vectors (the
    paper's comparison), "vertex" each vertex divergence on its own."""
    torch = _torch()
    if mode not in MC_MODES:
        raise ValueError(f"mode must be one of {sorted(MC_MODES)}")
    ptrs, ny, nx, dt = _moment_ptrs(mean_u, var_u, mean_v, var_v)
    iso, ip = _iso_arr(isovalues)
    if out is None:
        out = torch.empty((iso.size, ny - 1, nx - 1), dtype=torch.float32, device=mean_u.device)
    po = _dev(out, "out", (iso.size, ny - 1, nx - 1), torch.float32)
    _check(lib().pdiv_mc_lcp(*ptrs, dt, ny, nx, dx, dy, ip, iso.size, n_samples,
                             seed & 0xFFFFFFFFFFFFFFFF, MC_MODES[mode], po, _stream()))
    return out


def mc_sample_field(mean_u, var_u, mean_v, var_v, sample: int, seed: int):
    """Sample `sample` of the uncertain field as the MC draws it: (U, V) float32."""
    torch = _torch()
    ptrs, ny, nx, dt = _moment_ptrs(mean_u, var_u, mean_v, var_v)
    us = torch.empty((ny, nx), dtype=torch.float32, device=mean_u.device)
    vs = torch.empty_like(us)
    _check(lib().pdiv_mc_sample_field(*ptrs, dt, ny, nx, sample, seed & 0xFFFFFFFFFFFFFFFF,
                                      _p(us.data_ptr()), _p(vs.data_ptr()), _stream()))
    return us, vs


class Batch:
    """Many fields of uneven size in one persistent launch (optionally graph-replayed).

    fields: sequence of dicts with mean_u, var_u, mean_v, var_v (device planes of one
    dtype), isovalues (device float32 tensor, 1..16 values), dx, dy, and optionally
    lcp (device output [K][ny-1][nx-1], dense or a row-padded view; allocated
    row-padded (empty_lcp) if absent)."""

    GRAPH = 1
    AUTOTUNE = 2

    def __init__(self, fields: Sequence[dict], graph: bool = True, autotune: bool = False):
        torch = _torch()
        arr = (_Field * len(fields))()
        self.fields = []
        dt = None
        for k, f in enumerate(fields):
            ptrs, ny, nx, d = _moment_ptrs(f["mean_u"], f["var_u"], f["mean_v"], f["var_v"])
            dt = d if dt is None else dt
            if d != dt:
                raise ValueError("all fields of a batch share one dtype")
            iso = f["isovalues"]
            _dev(iso, "isovalues", None, torch.float32)
            out = f.get("lcp")
            if out is None:  # rows on 128-byte lines, so either tile layout may run
                out = empty_lcp(iso.numel(), ny, nx, device=f["mean_u"].device)
            po, pitch, plane = _lcp_out(out, iso.numel(), ny, nx)
            arr[k] = _Field(ptrs[0], ptrs[1], ptrs[2], ptrs[3], ny, nx,
                            float(f.get("dx", 1.0)), float(f.get("dy", 1.0)),
                            _p(iso.data_ptr()), iso.numel(), po, pitch, plane)
            self.fields.append(dict(f, lcp=out))
        flags = (self.GRAPH if graph else 0) | (self.AUTOTUNE if autotune else 0)
        h = _p()
        _check(lib().pdiv_batch_create(arr, len(fields), dt or 0, flags, _stream(), _c.byref(h)))
        self._h = h

    def launch(self):
        _check(lib().pdiv_batch_launch(self._h, _stream()))

    def info(self):
        a, b, c = _i32(), _i32(), _i64()
        _check(lib().pdiv_batch_info(self._h, _c.byref(a), _c.byref(b), _c.byref(c)))
        return dict(band_rows=a.value, strip_cells=b.value, n_tiles=c.value)

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().pdiv_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_plane(a):
    """A host plane as (contiguous array, dtype code): numpy float32 or
    float16, or a torch CPU tensor of float32, float16 or bfloat16 (passed
    as its raw 16-bit words)."""
    if hasattr(a, "is_cuda"):  # torch tensor
        if a.is_cuda:
            raise ValueError("put_field takes host planes, not device tensors")
        code = _dtype_code(a)
        a = a.contiguous()
        return (a.view(_torch().int16).numpy() if code == 2 else a.numpy()), code
    a = np.ascontiguousarray(a)
    codes = {np.dtype(np.float32): 0, np.dtype(np.float16): 1}
    if a.dtype not in codes:
        raise TypeError(f"unsupported host dtype {a.dtype}; use float32 or float16 "
                        "(bfloat16 as a torch CPU tensor)")
    return a, codes[a.dtype]


class Server:
    """Continuous-batching LCP server over device-resident fields.

    The binding remembers each field's grid, so that submit_lcp can check the
    output tensor: the C call takes no size for it and writes
    n_iso*(ny-1)*(nx-1) floats."""

    def __init__(self, hbm_budget: int, n_streams: int = 2):
        h = _p()
        _check(lib().pdiv_server_create(hbm_budget, n_streams, _c.byref(h)))
        self._h = h
        self._grid = {}

    def put_field(self, fid: int, mean_u, var_u, mean_v, var_v, dx=1.0, dy=1.0) -> int:
        """Host planes [ny][nx] of one dtype and shape (numpy float32/float16,
        or torch CPU float32/float16/bfloat16) -> ticket.  The planes are
        copied before the call returns."""
        planes = [_host_plane(a) for a in (mean_u, var_u, mean_v, var_v)]
        arrs = [a for a, _ in planes]
        code = planes[0][1]
        if arrs[0].ndim != 2:
            raise ValueError(f"mean_u must be a [ny][nx] plane, got shape {arrs[0].shape}")
        for (a, c), name in zip(planes[1:], ("var_u", "mean_v", "var_v")):
            if c != code or a.shape != arrs[0].shape:
                raise ValueError(f"{name} must match mean_u's shape {arrs[0].shape} and dtype")
        ny, nx = arrs[0].shape
        t = _u64()
        _check(lib().pdiv_server_put_field(self._h, fid, *[_p(a.ctypes.data) for a in arrs],
                                           code, ny, nx, dx, dy, _c.byref(t)))
        self._grid[fid] = (ny, nx)
        return t.value

    def reserve_staging(self, max_points: int, count: int, dtype=np.float32):
        """Pre-allocate and touch `count` pinned staging buffers for fields of up
        to max_points points."""
        code = {np.dtype(np.float32): 0, np.dtype(np.float16): 1}[np.dtype(dtype)]
        _check(lib().pdiv_server_reserve_staging(self._h, max_points, code, count))

    def submit_lcp(self, fid: int, isovalues, out, sync: bool = True) -> int:
        """Slider request: LCP maps of resident field fid at the isovalues into
        out, a contiguous float32 device tensor [n_iso][ny-1][nx-1] that must
        stay alive until the ticket completes.  The server writes it from its
        own streams, so work still pending on out in torch's current stream
        must finish first: with sync (the default) the current stream is
        synchronised before the request is submitted; pass sync=False only
        when no work on out can be pending."""
        iso, ip = _iso_arr(isovalues)
        grid = self._grid.get(fid)
        if grid is None:
            raise PdivError(1, f"field id {fid} was never put on this server")
        ny, nx = grid
        _dev(out, "out", (iso.size, ny - 1, nx - 1), _torch().float32)
        if sync:
            _torch().cuda.current_stream().synchronize()
        t = _u64()
        _check(lib().pdiv_server_submit_lcp(self._h, fid, ip, iso.size, _p(out.data_ptr()),
                                            _c.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1) -> int:
        r = _c.c_int()
        st = lib().pdiv_server_wait(self._h, ticket, timeout_us, _c.byref(r))
        _check(st)
        return r.value

    def poll(self, ticket: int):
        """The request's own status (0 = done) once it has finished, which
        retires the ticket like wait(); None while it is still running."""
        r = _c.c_int()
        st = lib().pdiv_server_wait(self._h, ticket, 0, _c.byref(r))
        if st == _TIMEOUT:
            return None
        _check(st)
        return r.value

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().pdiv_server_stats(self._h, _c.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().pdiv_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
