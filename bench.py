"""Throughput of the closed-form probabilistic-divergence path on one MI355X.

Workload (the size the throughput target is quoted on): an 8192x8192 field
whose mean and variance of U and V are stored in float32, 16 isovalues at
divergence quantiles 1%..99%.  One step = one pass of the closed-form hot path
over that input: Eq. 2-3 divergence Gaussians and the level-crossing
probability for all 16 isovalues, fused in one kernel (the field is read once,
16 LCP maps are written).  Inputs are resident in HBM before timing starts.

Besides the timed steps the run reports, on the same JSON line:
  roofline      algorithmic bytes of the fused kernel / its event-timed
                average duration, against 8 TB/s
  mc            the Monte Carlo comparison on the same field (1000 samples)
  legs          the other steps of the path timed alone (ensemble fit on the
                721x1440x50 ensemble, the two-step divergence + LCP, 16-bit
                storage)
  cpu_baseline  the FP64 oracle on a band of the same field, on this host,
                with the GPU-vs-oracle error on that band

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LCP cells/sec & % HBM peak (closed form vs GPU MC) at ≤1e-5 LCP abs err"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "lcp_fused_8192x8192_k16_f32_traffic.txt")
KERNEL_SRC = [os.path.join(ROOT, "paper_2510_01190_amd", "csrc", f)
              for f in ("k_lcp.hip", "pdiv_device.hpp")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SRC:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, or None if absent or taken on other kernel source."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    vals = {}
    for line in open(PROFILE_TRAFFIC):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_launches(fn, n, torch):
    """Average device time of fn() over n back-to-back launches, HIP events on
    the current stream (the stream every launch is enqueued on)."""
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(n):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / n / 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-legs", action="store_true")
    ap.add_argument("--no-mc", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mc-samples", type=int, default=1000)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the path is single-GPU in this build "
              "(multi-GPU sharding is a design note only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2510_01190_amd as P
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    P.lib()  # fail loudly if the library is missing

    log("generating the 8192x8192 field (seeded)")
    c3 = synth.config_c3()
    ny, nx = c3["ny"], c3["nx"]
    iso = c3["isovalues"]
    K = int(iso.size)
    mom = [torch.from_numpy(c3[k]).float().cuda() for k in ("mean_u", "var_u", "mean_v", "var_v")]
    cells = (ny - 1) * (nx - 1)
    out = torch.empty((K, ny - 1, nx - 1), dtype=torch.float32, device="cuda")

    def step():
        P.lcp_from_moments(*mom, iso, out=out)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(f"timing {args.steps} steps")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([a.elapsed_time(b) / 1e3 for a, b in evs])
    step_s = wall / args.steps
    kern_s = float(per.mean())
    value = cells * K / step_s
    alg_bytes = 4 * 4 * ny * nx + 4 * K * cells
    achieved = alg_bytes / kern_s / 1e9
    traffic = read_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": "lcp_kernel<16,true,float> (fused Eq. 2-3 + LCP)",
                "algorithmic_bytes_per_launch": alg_bytes,
                "kernel_ms_mean": round(kern_s * 1e3, 4),
                "kernel_ms_min": round(float(per.min()) * 1e3, 4)}
    log(f"step {step_s * 1e3:.3f} ms, kernel {kern_s * 1e3:.3f} ms, {achieved:.0f} GB/s")

    result = {"metric": METRIC, "value": round(value, 1), "unit": "LCP cells/s",
              "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "ms_per_step": round(step_s * 1e3, 4), "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
              "config": {"workload": "lcp_from_moments_8192x8192_k16_f32", "ny": ny, "nx": nx,
                         "n_iso": K, "storage": "float32", "cells": cells,
                         "path": "fused divergence Gaussian (Eq. 2-3) + closed-form LCP",
                         "parallelism": "single GPU"},
              "roofline": roofline}

    if not args.no_mc:
        S = args.mc_samples
        log(f"Monte Carlo comparison, {S} samples")
        mc_out = torch.empty_like(out)
        P.mc_lcp(*mom, iso, n_samples=2, seed=1, out=mc_out)
        torch.cuda.synchronize()
        t = time_launches(lambda: P.mc_lcp(*mom, iso, n_samples=S, seed=2025, out=mc_out), 1, torch)
        result["mc"] = {"value": round(cells * K / t, 1), "unit": "LCP cells/s", "samples": S,
                        "ms": round(t * 1e3, 3),
                        "point_samples_per_s": round(ny * nx * S / t, 1),
                        "closed_form_speedup": round(t / kern_s, 1)}
        d = (mc_out - out).double()
        result["mc"]["sse_vs_closed_form_per_map"] = round(float((d * d).sum()) / K, 3)
        del mc_out, d
        torch.cuda.empty_cache()

    if not args.no_legs:
        legs = {}
        dm = torch.empty((ny, nx), device="cuda")
        dv = torch.empty_like(dm)
        out2 = torch.empty_like(out)

        def two_step():
            P.lib().pdiv_divergence_gaussian(*[P._p(t.data_ptr()) for t in mom], 0, ny, nx, 1.0,
                                             1.0, P._p(dm.data_ptr()), P._p(dv.data_ptr()),
                                             P._stream())
            P.lcp(dm, dv, iso, out=out2)

        two_step()
        t = time_launches(two_step, 5, torch)
        legs["two_step_divergence_then_lcp_f32"] = {"ms": round(t * 1e3, 4),
                                                   "cells_per_s": round(cells * K / t, 1)}
        assert torch.equal(out, out2), "two-step path differs from the fused path"
        del out2, dm, dv
        for name, dt, bpe in (("f16", torch.float16, 2), ("bf16", torch.bfloat16, 2)):
            m16 = [torch.from_numpy(c3[k]).to(dt).cuda() for k in
                   ("mean_u", "var_u", "mean_v", "var_v")]
            P.lcp_from_moments(*m16, iso, out=out)
            t = time_launches(lambda: P.lcp_from_moments(*m16, iso, out=out), 10, torch)
            b = 4 * bpe * ny * nx + 4 * K * cells
            legs[f"fused_{name}_storage"] = {"ms": round(t * 1e3, 4),
                                             "cells_per_s": round(cells * K / t, 1),
                                             "achieved_GBs": round(b / t / 1e9, 1)}
            del m16
        step()  # restore the float32 maps for the accuracy sample below
        torch.cuda.synchronize()
        log("ensemble fit leg (721x1440, 50 members)")
        c2 = synth.config_c2()
        u = torch.from_numpy(c2["u_members"]).cuda()
        v = torch.from_numpy(c2["v_members"]).cuda()
        outs = [torch.empty((721, 1440), device="cuda") for _ in range(4)]

        def fit():
            P.lib().pdiv_moments(P._p(u.data_ptr()), P._p(v.data_ptr()), 0, 50, 721, 1440, 0, 1,
                                 *[P._p(o.data_ptr()) for o in outs], 0, P._stream())

        fit()
        t = time_launches(fit, 10, torch)
        b = 2 * 50 * 721 * 1440 * 4 + 4 * 4 * 721 * 1440
        legs["moments_721x1440_m50_f32"] = {"ms": round(t * 1e3, 4),
                                            "achieved_GBs": round(b / t / 1e9, 1),
                                            "frac_hbm": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}
        c2out = torch.empty((8, 720, 1439), device="cuda")
        t = time_launches(lambda: (fit(), P.lcp_from_moments(*outs, c2["isovalues"], out=c2out)),
                          10, torch)
        legs["pipeline_fit_then_lcp_721x1440_m50_k8"] = {"ms": round(t * 1e3, 4),
                                                        "cells_per_s": round(720 * 1439 * 8 / t, 1)}
        del u, v, outs, c2out
        result["legs"] = legs

    if not args.no_cpu_baseline:
        import oracle as O

        rows = (3328, 4864)
        log(f"CPU baseline: FP64 oracle on cell rows {rows[0]}..{rows[1]} (1 thread)")
        stored = [t.double().cpu().numpy() for t in mom]
        t_cpu = 0.0
        n_cpu = 0
        worst = 0.0
        for j0 in range(rows[0], rows[1], 256):
            j1 = min(j0 + 256, rows[1])
            a, b = j0 - 1, j1 + 2
            t = time.perf_counter()
            m, vv = O.divergence_gaussian(*[x[a:b] for x in stored], 1.0, 1.0)
            ref = O.lcp(m[1:-1], vv[1:-1], iso)
            t_cpu += time.perf_counter() - t
            n_cpu += ref.size
            g = out[:, j0:j1, :].double().cpu().numpy()
            worst = max(worst, float(np.max(np.abs(g - ref))))
        result["cpu_baseline"] = {"value": round(n_cpu / t_cpu, 1), "unit": "LCP cells/s",
                                  "cores": 1, "kind": "oracle",
                                  "sample": f"cell rows {rows[0]}-{rows[1] - 1} of the same "
                                            f"8192x8192 field, all {K} isovalues "
                                            f"({n_cpu} LCP values, {t_cpu:.1f} s, numpy float64)",
                                  "gpu_speedup": round(value / (n_cpu / t_cpu), 1),
                                  "gpu_max_abs_err_on_sample": worst}
        result["accuracy"] = {"max_abs_err_vs_fp64_oracle": worst, "bar": 1e-5,
                              "within_bar": worst <= 1e-5}

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
