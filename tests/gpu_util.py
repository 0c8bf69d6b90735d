"""Helpers for the GPU parity tests: device transfer and error summaries."""

import numpy as np
import torch

U32 = 2.0 ** -24  # unit roundoff of float32

TORCH_DT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def dev(a, dt="f32"):
    """float64 numpy -> device tensor of the storage dtype (round to nearest even)."""
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(TORCH_DT[dt]).cuda()


def host64(t):
    """Device tensor -> float64 numpy, exactly (every storage dtype upcasts exactly)."""
    return t.float().cpu().numpy().astype(np.float64)


def moments_dev(f, dt="f32"):
    return [dev(f[k], dt) for k in ("mean_u", "var_u", "mean_v", "var_v")]


def stored64(ts):
    return [host64(t) for t in ts]


def err_report(got, ref):
    d = np.abs(np.asarray(got, np.float64) - ref)
    return dict(max_abs=float(np.nanmax(d)) if d.size else 0.0,
                mean_abs=float(np.nanmean(d)) if d.size else 0.0)
