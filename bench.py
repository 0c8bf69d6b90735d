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
import ctypes
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
              for f in ("k_lcp.hip", "lcp_tile.hpp", "pdiv_device.hpp", "tail_coeffs.hpp")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(paths):
    """sha256 (first 16 hex digits) of source files with their comments
    removed and whitespace collapsed: counters taken on a kernel stay valid
    when only its comments or layout change, and go stale with any change to
    its code."""
    import re
    h = hashlib.sha256()
    for p in paths:
        text = open(p).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def kernel_hash():
    return source_hash(KERNEL_SRC)


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


def host_cpu():
    """CPU model and the number of CPUs this process may run on."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": name, "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_workers():
    """Worker processes for the all-cores CPU legs: the CPUs this process may
    run on, at most 16 (one GPU's share of the host)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _warm(_):
    import numpy  # noqa: F401
    import oracle  # noqa: F401
    return os.getpid()


def _shared_rows(task):
    from multiprocessing import shared_memory
    import numpy as np
    shm = shared_memory.SharedMemory(name=task[0])
    arr = np.ndarray(task[1], np.float64, buffer=shm.buf)
    return shm, [arr[q, task[2]:task[3]] for q in range(4)]


def _oracle_band(task):
    """Closed-form oracle on moment rows [a, b) of the shared float64 copy
    (cell rows a+1 .. b-2); returns (LCP values, seconds)."""
    import oracle as O
    shm, planes = _shared_rows(task)
    t = time.perf_counter()
    m, vv = O.divergence_gaussian(*planes, 1.0, 1.0)
    n = O.lcp(m[1:-1], vv[1:-1], task[4]).size
    dt = time.perf_counter() - t
    del planes, m, vv
    shm.close()
    return n, dt


def _mc_band(task):
    """Vector-level Monte Carlo oracle on moment rows [a, b) of the shared
    copy, as a field of its own; returns (LCP values, seconds)."""
    import oracle as O
    shm, planes = _shared_rows(task)
    t = time.perf_counter()
    n = O.mc_lcp(*planes, 1.0, 1.0, task[4], task[5], task[6]).size
    dt = time.perf_counter() - t
    del planes
    shm.close()
    return n, dt


def cpu_legs(stored, iso, rows, mc_rows=34, mc_samples=100, mc_target=1000):
    """CPU legs beside the single-thread oracle: the same oracle on the same
    cell rows spread over cpu_workers() processes, and the vector-level
    Monte Carlo oracle (mc_samples samples on mc_rows-row bands, scaled
    linearly to mc_target samples) on one core and on all workers.  The
    oracle is unchanged; the processes only split the rows."""
    import multiprocessing
    from multiprocessing import shared_memory
    import numpy as np
    ny, nx = stored[0].shape
    nw = cpu_workers()
    lo, hi = rows[0] - 1, rows[1] + 2
    mc_lo = lo  # Monte Carlo bands start at the top of the shared rows
    assert mc_lo + nw * mc_rows <= hi
    shape = (4, hi - lo, nx)
    shm = shared_memory.SharedMemory(create=True, size=8 * 4 * (hi - lo) * nx)
    out = {}
    try:
        arr = np.ndarray(shape, np.float64, buffer=shm.buf)
        for q in range(4):
            arr[q] = stored[q][lo:hi]
        del arr
        mc_task = lambda i: (shm.name, shape, i * mc_rows, (i + 1) * mc_rows, iso, mc_samples,
                             2025 + i)
        log(f"CPU Monte Carlo oracle, 1 thread ({mc_rows}x{nx} band, {mc_samples} samples)")
        n1, t1 = _mc_band(mc_task(0))
        scale = mc_target / mc_samples
        ctx = multiprocessing.get_context("spawn")
        with ctx.Pool(nw) as pool:
            pool.map(_warm, range(4 * nw))  # start-up and imports outside the clock
            log(f"CPU oracle on {nw} processes")
            tasks = [(shm.name, shape, j0 - 1 - lo, min(j0 + 256, rows[1]) + 2 - lo, iso)
                     for j0 in range(rows[0], rows[1], 256)]
            t = time.perf_counter()
            res = pool.map(_oracle_band, tasks, chunksize=1)
            wall = time.perf_counter() - t
            n_all = sum(r[0] for r in res)
            out["oracle_all_cores"] = {
                "value": round(n_all / wall, 1), "unit": "LCP cells/s", "cores": nw,
                "kind": "oracle", "sample": f"the same cell rows in {len(tasks)} bands of 256 "
                                            f"rows over {nw} processes ({wall:.2f} s wall)"}
            log(f"CPU Monte Carlo oracle on {nw} processes")
            t = time.perf_counter()
            res = pool.map(_mc_band, [mc_task(i) for i in range(nw)], chunksize=1)
            wall_mc = time.perf_counter() - t
        n_mc = sum(r[0] for r in res)
        sample = (f"{mc_rows}x{nx}-vertex bands of the same field, {len(iso)} isovalues, "
                  f"{mc_samples} samples, time scaled x{scale:g} to {mc_target} samples")
        out["mc_1core"] = {"value": round(n1 / (t1 * scale), 1),
                           "unit": f"LCP cells/s at {mc_target} samples", "cores": 1,
                           "kind": "oracle (vector-level Monte Carlo, numpy float64)",
                           "sample": f"one band; {sample} ({t1:.1f} s)",
                           "point_samples_per_s": round(mc_rows * nx * mc_samples / t1, 1)}
        out["mc_all_cores"] = {"value": round(n_mc / (wall_mc * scale), 1),
                               "unit": f"LCP cells/s at {mc_target} samples", "cores": nw,
                               "kind": "oracle (vector-level Monte Carlo, numpy float64)",
                               "sample": f"{nw} bands; {sample} ({wall_mc:.1f} s wall)"}
    finally:
        shm.close()
        shm.unlink()
    return out


PROFILE_MC = os.path.join(ROOT, "profiles", "mc_8192x8192_k16_s1000_valu.txt")
MC_SRC = [os.path.join(ROOT, "paper_2510_01190_amd", "csrc", f)
          for f in ("k_mc.hip", "mc_rank.hpp", "pdiv_device.hpp")]


def read_mc_valu():
    """(fraction of the class-weighted vector-ALU issue bound, VALU wave
    instructions per point-sample) of the Monte Carlo kernel from the
    committed counter summary, or None if absent or taken on other kernel
    source."""
    if not os.path.exists(PROFILE_MC):
        return None
    vals = {}
    for line in open(PROFILE_MC):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != source_hash(MC_SRC):
        return None
    try:
        return (float(vals["alu_bound_frac"]),
                float(vals["valu_wave_instructions_per_point_sample"]))
    except (KeyError, ValueError):
        return None


def guarded(name, fn, *args, **kw):
    """Run an optional leg; a failure is logged and recorded in its entry so
    that the headline line is still printed."""
    try:
        return fn(*args, **kw)
    except Exception as e:  # noqa: BLE001 -- any failure of a side leg
        log(f"{name} failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}


def time_launches(fn, n, torch, settle_s=0.15):
    """Average device time of fn() over n back-to-back launches, HIP events on
    the current stream (the stream every launch is enqueued on), after fn()
    has run back to back for settle_s seconds (see settle), so that each leg,
    like the headline step, is timed at settled clocks."""
    if settle_s > 0:
        settle(fn, torch, settle_s)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(n):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / n / 1e3


SETTLE_S = 0.4


def settle(fn, torch, seconds=SETTLE_S):
    """Run fn() back to back for `seconds` of wall time before anything is
    timed.  Under sustained load the MI355X's clocks take tens of
    milliseconds to settle: measured per dispatch, the first ~20 launches of
    the 8192^2 fused step take 1.10-1.43 ms and later ones 1.06-1.07 ms.
    Without this, a few warmup steps leave the timed steps in that ramp."""
    import time as _t
    t0 = _t.perf_counter()
    n = 0
    while _t.perf_counter() - t0 < seconds:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()
        n += 8
    return n


def batch_leg(P, synth, torch, np):
    """512 fields of uneven size (sides log-uniform in [64, 2048]), 4 isovalues
    each: one persistent launch (autotuned, graph-replayed) against 512
    separate fused launches on one stream."""
    log("batch leg: generating 512 fields")
    F = synth.config_c4()
    fields, outs_pf = [], []
    for f in F:
        d = {k: torch.from_numpy(f[k]).float().cuda() for k in ("mean_u", "var_u", "mean_v", "var_v")}
        d["isovalues"] = torch.from_numpy(f["isovalues"]).cuda()
        d["iso_host"] = f["isovalues"]
        fields.append(d)
        outs_pf.append(P.empty_lcp(4, f["ny"], f["nx"]))
    cells = sum(4 * (f["ny"] - 1) * (f["nx"] - 1) for f in F)
    in_bytes = sum(16 * f["ny"] * f["nx"] for f in F)

    def per_field():
        for d, o in zip(fields, outs_pf):
            P.lcp_from_moments(d["mean_u"], d["var_u"], d["mean_v"], d["var_v"], d["iso_host"], out=o)

    per_field()
    t_pf = time_launches(per_field, 3, torch)
    log("batch leg: autotuning the persistent launch")
    plain = P.Batch(fields, graph=False)
    plain.launch()
    t_plain = time_launches(plain.launch, 10, torch)
    b = P.Batch(fields, graph=True, autotune=True)
    b.launch()
    t_b = time_launches(b.launch, 10, torch)
    torch.cuda.synchronize()
    same = all(torch.equal(o, g["lcp"]) for o, g in zip(outs_pf, b.fields))
    info = b.info()
    plain.close()
    b.close()
    return {"fields": len(F), "lcp_values": cells,
            "per_field_launches_ms": round(t_pf * 1e3, 3),
            "batch_ms": round(t_plain * 1e3, 3),
            "batch_graph_autotuned_ms": round(t_b * 1e3, 3),
            "speedup_vs_per_field": round(t_pf / t_b, 2),
            "cells_per_s": round(cells / t_b, 1),
            "achieved_GBs": round((in_bytes + 4 * cells) / t_b / 1e9, 1),
            "tile": info, "bitwise_equal_to_per_field": bool(same)}


def volume_leg(P, synth, torch, np, n=512):
    """The 3D extension on an n^3 float32 field (six moment volumes): the
    divergence Gaussian with the z term, then the 8-corner LCP at 1, 4 and
    16 isovalues, and the two fused, each against its algorithmic bytes;
    the maps of sampled cell layers against the oracle, and the oracle's own
    rate on one slab."""
    import oracle as O
    log(f"3D leg: generating the {n}^3 field (seeded)")
    keys = ("mean_u", "var_u", "mean_v", "var_v", "mean_w", "var_w")
    f = synth.gen_moments_3d(n, n, n, synth.SEED_BASE + 30, dtype=np.float32)
    ts = [torch.from_numpy(f[k]).cuda() for k in keys]

    def oracle_vertices(k0):
        # the oracle's divergence Gaussians of vertex planes k0..k0+2 from the
        # stored volumes' z slab k0-1..k0+3 (differenced as in the whole volume)
        a, b = max(0, k0 - 1), min(n, k0 + 4)
        m, v = O.divergence_gaussian_3d(*[f[k][a:b].astype(np.float64) for k in keys],
                                        1.0, 1.0, 1.0)
        return m[k0 - a:k0 - a + 3], v[k0 - a:k0 - a + 3]

    slabs = {k0: oracle_vertices(k0) for k0 in (0, n // 2 - 2, n - 3)}
    del f
    pts = n ** 3
    cells = (n - 1) ** 3
    dm, dv = P.divergence_gaussian_3d(*ts)
    t = time_launches(lambda: P.divergence_gaussian_3d(*ts), 10, torch)
    b = 6 * 4 * pts + 2 * 4 * pts
    out = {"grid": [n, n, n], "storage": "float32",
           "divergence_3d": {"ms": round(t * 1e3, 4), "algorithmic_bytes": b,
                             "achieved_GBs": round(b / t / 1e9, 1),
                             "frac_hbm": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}}
    sub = slabs[n // 2 - 2][0]

    def timed(fn, b, k):
        fn()
        t = time_launches(fn, 10, torch)
        return {"ms": round(t * 1e3, 4), "cells_per_s": round(k * cells / t, 1),
                "algorithmic_bytes": b, "achieved_GBs": round(b / t / 1e9, 1),
                "frac_hbm": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}

    for k in (1, 4, 16):
        iso = np.quantile(sub, np.linspace(0.2, 0.8, k) if k > 1 else [0.5]).astype(np.float32)
        b2 = 8 * pts + 4 * k * cells    # two-step LCP: divergence volumes in, maps out
        bf = 6 * 4 * pts + 4 * k * cells  # fused: the six moment volumes in
        # rows padded to 512 floats (whole-line stores: the 64-cell tile with
        # the seam step), then dense [K][511][511][511] rows (63-cell tile)
        for name, make in (("", lambda: P.empty_lcp_3d(k, n, n, n)),
                           ("_dense", lambda: torch.empty((k, n - 1, n - 1, n - 1),
                                                          device="cuda"))):
            o = make()
            leg = timed(lambda: P.lcp_3d(dm, dv, iso, out=o), b2, k)
            if k == 4:
                worst = 0.0
                for k0, (m, v) in slabs.items():
                    tc = time.perf_counter()
                    r = O.lcp_3d(m, v, iso)
                    tc = time.perf_counter() - tc
                    worst = max(worst, float(np.max(np.abs(
                        o[:, k0:k0 + 2].double().cpu().numpy() - r))))
                leg["max_abs_err_vs_fp64_oracle_sampled_layers"] = worst
                leg["cpu_oracle_cells_per_s_1core"] = round(r.size / tc, 1)
                if not name:
                    out["two_step_k4_ms"] = round(out["divergence_3d"]["ms"] + leg["ms"], 4)
            out[f"lcp_3d_k{k}{name}"] = leg
            # the two steps fused: the divergence volumes never reach HBM
            out[f"fused_3d_k{k}{name}"] = timed(lambda: P.lcp_3d_from_moments(*ts, iso, out=o),
                                                bf, k)
            del o
    del dm, dv, ts
    return out


LCP_BIN_EDGES = [0.0, 1e-6, 1e-3, 0.5, 1 - 1e-3, 1 - 1e-6, 1.0 + 1e-12]
LCP_BIN_NAMES = ["[0,1e-6)", "[1e-6,1e-3)", "[1e-3,0.5)", "[0.5,1-1e-3)", "[1-1e-3,1-1e-6)",
                 "[1-1e-6,1]"]


def new_bins():
    """Per-bin error records of LCP maps against the oracle (see add_to_bins)."""
    out = []
    for q, nm in enumerate(LCP_BIN_NAMES):
        b = {"bin": nm, "count": 0, "max_abs": 0.0}
        if LCP_BIN_EDGES[q] < 0.5:
            b["max_rel"] = 0.0
        else:
            b["max_abs_in_ulps_of_1"] = 0.0
        out.append(b)
    return out


def add_to_bins(bins, ref, err, np):
    """Bins of the oracle value L: count and max abs error; below 0.5 also
    the max error relative to L (cells with L >= 1e-9: below that the
    oracle's literal 1 - A - B has no relative accuracy, its absolute error
    being ~1e-16); above 0.5 the max abs error in units of 2^-24, the
    spacing of float32 values below 1 (the finest a float32 map resolves
    1 - L)."""
    for q, b in enumerate(bins):
        sel = (ref >= LCP_BIN_EDGES[q]) & (ref < LCP_BIN_EDGES[q + 1])
        if not sel.any():
            continue
        b["count"] += int(sel.sum())
        b["max_abs"] = max(b["max_abs"], float(err[sel].max()))
        if "max_rel" in b:
            rs = sel & (ref >= 1e-9)
            if rs.any():
                b["max_rel"] = max(b["max_rel"], float((err[rs] / ref[rs]).max()))
        else:
            b["max_abs_in_ulps_of_1"] = round(b["max_abs"] / 2.0 ** -24, 3)


def near01_leg(P, synth, torch, np, rows=(4096, 4224)):
    """LCP error near 0 and 1 in the headline launch (fused Eq. 2-3 + LCP, 16
    isovalues, rows padded to 128-byte lines and interleaved by isovalue) on
    the precision sweep's grid with a small spread, sigma ~ U[0.002, 0.02],
    whose cells sit deep in the tails or are crossed with near certainty.
    Per storage type and per bin of the oracle value: count, max abs error,
    and below 0.5 the max error relative to L (cells with L >= 1e-9: below
    that the oracle's literal 1 - A - B has no relative accuracy, its
    absolute error being ~1e-16), above 0.5 the max abs error in units of
    2^-24 (the spacing of float32 values below 1, the finest a float32 map
    resolves 1 - L); against the FP64 oracle on the stored values (Eq. 2-3
    in float64)."""
    import oracle as O
    log("near-0/1 accuracy: generating the low-spread 8192x8192 field (seeded)")
    f = synth.config_c3_low_spread()
    ny, nx = f["ny"], f["nx"]
    iso = f["isovalues"]
    keys = ("mean_u", "var_u", "mean_v", "var_v")
    a0, a1 = rows
    out = P.empty_lcp(iso.size, ny, nx, interleave_rows=True)
    res = {"field": "8192x8192, sigma ~ U[0.002, 0.02], 16 isovalues at divergence quantiles "
                    "linspace(0.01, 0.99, 16)",
           "sample": f"cell rows {a0}-{a1 - 1}, all 16 isovalues",
           "launch": "fused, rows interleaved by isovalue, pitch 8192 (the headline's)"}
    for name, dt in (("f32", torch.float32), ("f16", torch.float16), ("bf16", torch.bfloat16)):
        ts = [torch.from_numpy(f[k]).to(dt).cuda() for k in keys]
        P.lcp_from_moments(*ts, iso, out=out)
        g = out[:, a0:a1, :].double().cpu().numpy()
        st = [t[a0 - 1:a1 + 2].double().cpu().numpy() for t in ts]
        del ts
        m, v = O.divergence_gaussian(*st, 1.0, 1.0)
        ref = O.lcp(m[1:-1], v[1:-1], iso)
        err = np.abs(g - ref)
        bins = new_bins()
        add_to_bins(bins, ref, err, np)
        res[name] = {"max_abs": float(err.max()), "mean_abs": float(err.mean()),
                     "bins_by_oracle_lcp": bins}
    del out
    torch.cuda.empty_cache()
    return res


def mc_leg(P, synth, torch, np, samples=1000):
    """The Monte Carlo comparison alone on the 8192x8192 field at 16
    isovalues (one launch after a short warmup launch)."""
    c3 = synth.config_c3()
    mom = [torch.from_numpy(c3[k]).float().cuda() for k in ("mean_u", "var_u", "mean_v", "var_v")]
    iso = c3["isovalues"]
    out = torch.empty((iso.size, c3["ny"] - 1, c3["nx"] - 1), device="cuda")
    P.mc_lcp(*mom, iso, n_samples=2, seed=1, out=out)
    t = time_launches(lambda: P.mc_lcp(*mom, iso, n_samples=samples, seed=2025, out=out), 1, torch,
                      settle_s=0)
    return {"ms": round(t * 1e3, 3), "samples": samples,
            "point_samples_per_s": round(c3["ny"] * c3["nx"] * samples / t, 1)}


def served_leg(P, synth, torch, np, n_streams=2, fracs=(0.5, 0.9), baseline=True):
    """Poisson request stream of 10^4 requests: 70% isovalue-slider requests
    (1-4 isovalues) on a field already resident on the device, 30% new float32
    square fields with sides log-uniform in [256, 4096] (rounded to whole
    points).  A new field of side s is the first s^2 values of each plane of
    one pre-generated 4096^2 field, viewed as [s][s] (no host copy before the
    call; for s < 4096 its rows are consecutive pieces of the big field's
    rows).  Capacity is measured with
    every request submitted at once; the stream then runs at 50% and 90% of
    it.  Clients are independent: new fields are put from two client threads
    (their host copy into pinned staging takes milliseconds), sliders from the
    main thread.  Latency is the server's, from each call to its result on the
    device; `call_lag` is how late each call started after its arrival time.
    The same requests handled one at a time with per-request launches, within
    the same HBM budget, give the baseline."""
    import time as _t
    from concurrent.futures import ThreadPoolExecutor
    log("served leg: preparing the 4096^2 field the new fields are cut from")
    big_side = 4096
    f = synth.gen_moments(big_side, big_side, synth.SEED_BASE + 5 + big_side,
                          n_features=big_side * big_side // 65536)
    big = [np.ascontiguousarray(f[k], np.float32).ravel()
           for k in ("mean_u", "var_u", "mean_v", "var_v")]
    del f

    def planes(side):  # zero-copy [side][side] views
        return [b[: side * side].reshape(side, side) for b in big]

    budget = 24 << 30
    n_req = 10000
    n_staging = 6
    n_put_threads = 2
    first_sides = (776, 2353)  # resident before the clock starts

    def stream(rate, seed):
        reqs = synth.request_stream(n_req, rate, seed)
        for r in reqs:
            if r["kind"] == "new":
                r["side"] = int(min(big_side, max(256, round(float(r["side"])))))
        return reqs

    # output ring: 8 buffers of the largest request's size, viewed per request
    n_ring = 8
    ring = [torch.empty(4 * (big_side - 1) ** 2, device="cuda") for _ in range(n_ring)]

    def ring_view(q, k, side):
        return ring[q][: k * (side - 1) ** 2].view(k, side - 1, side - 1)

    def pct(v, q):
        return round(float(np.percentile(np.asarray(v) * 1e6, q)), 1) if v else None

    def run(reqs, paced):
        srv = P.Server(hbm_budget=budget, n_streams=n_streams)
        # pinned staging set aside before the clock starts, as the one-at-a-time
        # baseline's runtime keeps its own staging buffers warm
        srv.reserve_staging(big_side ** 2, n_staging)
        ready = []    # (id, side) of fields whose upload has completed
        pending = []  # (id, side, future of the put_field ticket)
        tickets = []
        last = {}     # ring slot -> ticket of the slider writing it
        used = 0
        lag = {"slider": [], "new": []}
        failed_puts = 0
        next_id = 0
        # two fields resident before the clock starts so sliders have targets
        for s_ in first_sides:
            srv.wait(srv.put_field(next_id, *planes(s_)))
            ready.append((next_id, s_))
            next_id += 1
        puts = ThreadPoolExecutor(max_workers=n_put_threads)
        t0 = _t.perf_counter()

        def put(fid, side, t_arr):
            lag["new"].append(_t.perf_counter() - t0 - t_arr)
            return srv.put_field(fid, *planes(side))

        def refresh():
            nonlocal failed_puts
            keep = []
            for fid, side, fut in pending:
                if not fut.done():
                    keep.append((fid, side, fut))
                    continue
                try:
                    st = srv.poll(fut.result())
                except P.PdivError:
                    failed_puts += 1
                    continue
                if st is None:
                    keep.append((fid, side, fut))
                elif st == 0:
                    ready.append((fid, side))
                else:
                    failed_puts += 1
            pending[:] = keep

        for r in reqs:
            if paced:
                while _t.perf_counter() - t0 < r["t"]:
                    pass
            if r["kind"] == "new":
                side = r["side"]
                pending.append((next_id, side, puts.submit(put, next_id, side, r["t"])))
                next_id += 1
                continue
            refresh()
            iso = (r["iso_u"] - 0.5).astype(np.float32) * 0.05
            while True:
                while not ready:  # every resident field was evicted: wait for an upload
                    if not pending:
                        pending.append((next_id, 776, puts.submit(put, next_id, 776, r["t"])))
                        next_id += 1
                    refresh()
                fid, side = ready[int(r["pick"] * len(ready))]
                slot = used % n_ring
                if slot in last:  # the buffer's previous writer must be done
                    srv.wait(last.pop(slot))
                if paced:
                    lag["slider"].append(_t.perf_counter() - t0 - r["t"])
                try:
                    # no torch work ever touches the ring: nothing to order after
                    t = srv.submit_lcp(fid, iso, ring_view(slot, len(iso), side), sync=False)
                except P.PdivError:  # evicted since it was ready: pick another
                    ready.remove((fid, side))
                    if paced:
                        lag["slider"].pop()
                    continue
                used += 1
                last[slot] = t
                tickets.append(t)
                break
        for _, _, fut in pending:
            try:
                srv.wait(fut.result())
            except P.PdivError:
                failed_puts += 1
        puts.shutdown()
        for t in tickets:
            try:
                srv.wait(t)
            except P.PdivError:  # already waited on when its ring slot was reused
                pass
        wall = _t.perf_counter() - t0
        st = srv.stats()
        srv.close()
        st["failed_puts"] = failed_puts
        st["lag"] = lag
        return wall, st

    reqs = stream(1e9, 11)  # back to back: capacity
    wall, st = run(reqs, paced=False)
    capacity = n_req / wall
    out = {"requests": n_req, "budget_bytes": budget, "n_streams": n_streams,
           "client_put_threads": n_put_threads,
           "pinned_staging": f"{n_staging} x {16 * big_side ** 2} B reserved before timing",
           "new_field_sides": "log-uniform in [256, 4096], rounded; each new field is the "
                              "first side^2 values of a 4096^2 field's planes viewed as "
                              "[side][side]",
           "capacity_req_per_s": round(capacity, 1),
           "capacity_lcp_cells_per_s": round(st["lcp_cells"] / wall, 1)}
    for frac in fracs:
        rate = frac * capacity
        log(f"served leg: Poisson stream at {int(frac * 100)}% of capacity")
        wall, st = run(stream(rate, 12), paced=True)
        lag = st["lag"]
        out[f"at_{int(frac * 100)}pct"] = {
            "rate_req_per_s": round(rate, 1), "failed": st["failed"] + st["failed_puts"],
            "p50_us": round(st["p50_us"], 1), "p99_us": round(st["p99_us"], 1),
            "p50_slider_us": round(st["p50_slider_us"], 1),
            "p99_slider_us": round(st["p99_slider_us"], 1),
            "p50_new_us": round(st["p50_new_us"], 1), "p99_new_us": round(st["p99_new_us"], 1),
            "call_lag_p50_p99_slider_us": [pct(lag["slider"], 50), pct(lag["slider"], 99)],
            "call_lag_p50_p99_new_us": [pct(lag["new"], 50), pct(lag["new"], 99)],
            "launches": st["launches"], "peak_bytes": st["peak_bytes"],
            "throughput_req_per_s": round(n_req / wall, 1)}
    if not baseline:
        return out
    # baseline: the same back-to-back stream, one request at a time, keeping
    # fields resident within the same budget (oldest dropped first)
    log("served leg: one-request-at-a-time baseline")
    res = {}
    nid = 0
    for s_ in first_sides:
        ts = [torch.from_numpy(p).cuda() for p in planes(s_)]
        res[nid] = (P.divergence_gaussian(*ts), s_)
        nid += 1
    torch.cuda.synchronize()
    held = sum(8 * s_ * s_ for _, s_ in res.values())
    t0 = _t.perf_counter()
    order = list(res)
    for r in reqs:
        if r["kind"] == "new":
            side = r["side"]
            while held + 24 * side * side > budget:
                held -= 8 * res.pop(order.pop(0))[1] ** 2
            ts = [torch.from_numpy(p).cuda() for p in planes(side)]
            res[nid] = (P.divergence_gaussian(*ts), side)
            held += 8 * side * side
            del ts
            order.append(nid)
            nid += 1
        else:
            fid = order[int(r["pick"] * len(order))]
            (dm, dv), side = res[fid]
            iso = (r["iso_u"] - 0.5).astype(np.float32) * 0.05
            P.lcp(dm, dv, iso)
        torch.cuda.synchronize()
    base = _t.perf_counter() - t0
    del res
    out["one_at_a_time_req_per_s"] = round(n_req / base, 1)
    out["served_speedup_vs_one_at_a_time"] = round(capacity * base / n_req, 2)
    return out


def contour_timing(P, torch, dm, c):
    """pdiv_isocontour (count, row scan, write) on the divergence-mean plane
    dm at isovalue c, timed over 10 launches into a buffer sized by a first
    call."""
    ny, nx = dm.shape
    offs = torch.empty(ny, dtype=torch.int64, device="cuda")
    n_seg = int(P.isocontour(dm, c).shape[0])
    segs = torch.empty((max(n_seg, 1), 4), device="cuda")

    def contour():
        P.lib().pdiv_isocontour(P._p(dm.data_ptr()), ny, nx, ctypes.c_float(c),
                                P._p(offs.data_ptr()), P._p(segs.data_ptr()), n_seg,
                                P._stream())

    contour()
    t = time_launches(contour, 10, torch)
    b = 2 * 4 * ny * nx + 16 * n_seg + 16 * ny
    return {"ms": round(t * 1e3, 4), "segments": n_seg, "achieved_GBs": round(b / t / 1e9, 1),
            "frac_hbm": round(b / t / 1e9 / HBM_PEAK_GBS, 4),
            "note": "count pass, row scan and write pass; bytes = field read twice + segments"}


def c3_resident(synth, torch):
    """The 8192x8192 field's four float32 moment planes on the device, its
    isovalues and sizes."""
    c3 = synth.config_c3()
    mom = [torch.from_numpy(c3[k]).float().cuda() for k in ("mean_u", "var_u", "mean_v", "var_v")]
    return mom, c3["isovalues"], c3["ny"], c3["nx"]


def isocontour_leg(P, synth, torch, np):
    """The mean-field isocontour of the 8192x8192 field's divergence at its
    middle isovalue alone (for profiling the three contour kernels)."""
    mom, iso, ny, nx = c3_resident(synth, torch)
    dm = torch.empty((ny, nx), device="cuda")
    dv = torch.empty_like(dm)
    P.lib().pdiv_divergence_gaussian(*[P._p(t.data_ptr()) for t in mom], 0, ny, nx, 1.0, 1.0,
                                     P._p(dm.data_ptr()), P._p(dv.data_ptr()), P._stream())
    return contour_timing(P, torch, dm, float(iso[iso.size // 2]))


def dense_leg(P, synth, torch, np):
    """The fused kernel into dense [K][ny-1][nx-1] maps alone (for profiling
    that output layout)."""
    mom, iso, ny, nx = c3_resident(synth, torch)
    K = int(iso.size)
    cells = (ny - 1) * (nx - 1)
    dense = torch.empty((K, ny - 1, nx - 1), device="cuda")
    P.lcp_from_moments(*mom, iso, out=dense)
    t = time_launches(lambda: P.lcp_from_moments(*mom, iso, out=dense), 10, torch)
    b = 4 * 4 * ny * nx + 4 * K * cells
    return {"ms": round(t * 1e3, 4), "cells_per_s": round(cells * K / t, 1),
            "achieved_GBs": round(b / t / 1e9, 1), "frac_hbm": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-legs", action="store_true")
    ap.add_argument("--no-mc", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-legs", action="store_true",
                    help="only the single-thread oracle in the CPU baseline")
    ap.add_argument("--mc-samples", type=int, default=1000)
    ap.add_argument("--only-leg", choices=["volume_3d", "batch", "served", "mc", "near01", "isocontour",
                             "dense"],
                    help="run one leg alone and print its JSON (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library's path runs on one GPU "
              "(how it would shard over several is described, not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2510_01190_amd as P
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = 1 << 28  # 2^28 floats = 1 GiB read and 1 GiB written per copy
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}))
        return
    P.lib()  # fail loudly if the library is missing
    if args.only_leg:
        fn = {"volume_3d": volume_leg, "batch": batch_leg, "served": served_leg,
              "mc": mc_leg, "near01": near01_leg, "isocontour": isocontour_leg,
              "dense": dense_leg}[args.only_leg]
        print(json.dumps(fn(P, synth, torch, np)), flush=True)
        return

    log("generating the 8192x8192 field (seeded)")
    c3 = synth.config_c3()
    ny, nx = c3["ny"], c3["nx"]
    iso = c3["isovalues"]
    K = int(iso.size)
    mom = [torch.from_numpy(c3[k]).float().cuda() for k in ("mean_u", "var_u", "mean_v", "var_v")]
    cells = (ny - 1) * (nx - 1)
    # LCP maps viewed as [K][ny-1][nx-1]; each row is padded to a multiple of
    # 32 floats (8191 cells -> pitch 8192, 0.012% more memory), so every row
    # starts on a 128-byte line and every store writes whole lines, and row j
    # of the K maps are adjacent in memory (a [ny-1][K][8192] buffer), which
    # the fused kernel writes about 3% faster than K planes 256 MiB apart;
    # planar pitched and dense outputs are timed as legs
    out = P.empty_lcp(K, ny, nx, interleave_rows=True)
    pitch = out.stride(1)

    def step():
        P.lcp_from_moments(*mom, iso, out=out)

    n_settle = settle(step, torch)
    log(f"device settled with {n_settle} steps; warmup {args.warmup}")
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
                "traffic": traffic,
                "kernel": "lcp_kernel_paired<16,true,float> (fused Eq. 2-3 + LCP, "
                          "line-aligned rows, maps interleaved by rows)",
                "algorithmic_bytes_per_launch": alg_bytes,
                "kernel_ms_mean": round(kern_s * 1e3, 4),
                "kernel_ms_min": round(float(per.min()) * 1e3, 4)}
    log(f"step {step_s * 1e3:.3f} ms, kernel {kern_s * 1e3:.3f} ms, {achieved:.0f} GB/s")

    result = {"metric": METRIC, "value": round(value, 1), "unit": "LCP cells/s",
              "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "ms_per_step": round(step_s * 1e3, 4), "settle_steps": n_settle,
              "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
              "config": {"workload": "lcp_from_moments_8192x8192_k16_f32", "ny": ny, "nx": nx,
                         "n_iso": K, "storage": "float32", "cells": cells,
                         "output_row_pitch_floats": pitch,
                         "output_plane_stride_floats": out.stride(0),
                         "output_layout": "rows of the K maps interleaved ([ny-1][K][pitch])",
                         "path": "fused divergence Gaussian (Eq. 2-3) + closed-form LCP",
                         "parallelism": "single GPU"},
              "roofline": roofline}

    if not args.no_mc:
        S = args.mc_samples
        log(f"Monte Carlo comparison, {S} samples")
        mc_out = torch.empty((K, ny - 1, nx - 1), device="cuda")
        P.mc_lcp(*mom, iso, n_samples=2, seed=1, out=mc_out)
        torch.cuda.synchronize()
        t = time_launches(lambda: P.mc_lcp(*mom, iso, n_samples=S, seed=2025, out=mc_out), 1,
                          torch, settle_s=0)
        result["mc"] = {"value": round(cells * K / t, 1), "unit": "LCP cells/s", "samples": S,
                        "ms": round(t * 1e3, 3),
                        "point_samples_per_s": round(ny * nx * S / t, 1),
                        "closed_form_speedup": round(t / kern_s, 1)}
        valu = read_mc_valu()
        if valu is not None:
            frac, ipps = valu
            result["mc"]["roofline"] = {
                "bound": "alu", "achieved": frac, "peak": 1.0,
                "unit": "fraction of the vector-ALU issue bound: the launch's VALU instruction "
                        "counts per class times each class's measured cycles per instruction "
                        "per SIMD, over the launch's cycles (profiles/mc_8192x8192_k16_s1000_valu.txt)",
                "frac": frac, "valu_wave_instructions_per_point_sample": ipps}
        d = (mc_out - out).double()
        result["mc"]["sse_vs_closed_form_per_map"] = round(float((d * d).sum()) / K, 3)
        del mc_out, d
        torch.cuda.empty_cache()

    if not args.no_legs:
        legs = {}
        planar = P.empty_lcp(K, ny, nx)
        P.lcp_from_moments(*mom, iso, out=planar)
        t = time_launches(lambda: P.lcp_from_moments(*mom, iso, out=planar), 10, torch)
        legs["fused_f32_planar_pitched_output"] = {
            "ms": round(t * 1e3, 4), "cells_per_s": round(cells * K / t, 1),
            "achieved_GBs": round(alg_bytes / t / 1e9, 1),
            "bitwise_equal_to_headline": bool(torch.equal(planar, out))}
        del planar
        dense = torch.empty((K, ny - 1, nx - 1), device="cuda")
        P.lcp_from_moments(*mom, iso, out=dense)
        t = time_launches(lambda: P.lcp_from_moments(*mom, iso, out=dense), 10, torch)
        legs["fused_f32_dense_output_rows"] = {
            "ms": round(t * 1e3, 4), "cells_per_s": round(cells * K / t, 1),
            "achieved_GBs": round(alg_bytes / t / 1e9, 1),
            "bitwise_equal_to_headline": bool(torch.equal(dense, out))}
        del dense
        dm = torch.empty((ny, nx), device="cuda")
        dv = torch.empty_like(dm)
        out2 = P.empty_lcp(K, ny, nx, interleave_rows=True)

        def two_step():
            P.lib().pdiv_divergence_gaussian(*[P._p(t.data_ptr()) for t in mom], 0, ny, nx, 1.0,
                                             1.0, P._p(dm.data_ptr()), P._p(dv.data_ptr()),
                                             P._stream())
            P.lcp(dm, dv, iso, out=out2)

        two_step()
        t = time_launches(two_step, 5, torch)
        # each step alone: Eq. 2-3 (16 B read + 8 B written per point) and the
        # LCP from the divergence Gaussians (8 B read per point, 4 B per value)
        t_div = time_launches(lambda: P.lib().pdiv_divergence_gaussian(
            *[P._p(x.data_ptr()) for x in mom], 0, ny, nx, 1.0, 1.0, P._p(dm.data_ptr()),
            P._p(dv.data_ptr()), P._stream()), 10, torch)
        t_lcp = time_launches(lambda: P.lcp(dm, dv, iso, out=out2), 10, torch)
        b_div = 24 * ny * nx
        b_lcp = 8 * ny * nx + 4 * K * cells
        legs["two_step_divergence_then_lcp_f32"] = {
            "ms": round(t * 1e3, 4), "cells_per_s": round(cells * K / t, 1),
            "divergence_ms": round(t_div * 1e3, 4),
            "divergence_achieved_GBs": round(b_div / t_div / 1e9, 1),
            "divergence_frac_hbm": round(b_div / t_div / 1e9 / HBM_PEAK_GBS, 4),
            "lcp_from_divergence_ms": round(t_lcp * 1e3, 4),
            "lcp_from_divergence_achieved_GBs": round(b_lcp / t_lcp / 1e9, 1),
            "lcp_from_divergence_frac_hbm": round(b_lcp / t_lcp / 1e9 / HBM_PEAK_GBS, 4)}
        assert torch.equal(out, out2), "two-step path differs from the fused path"
        # the mean-field isocontour (marching squares) of the divergence at
        # the middle isovalue: count, scan and write, one call
        legs["isocontour_8192x8192_mean_field"] = contour_timing(P, torch, dm,
                                                                 float(iso[K // 2]))
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
        # the Red Sea pre-stage (Sec. 4) on the same ensemble: each member's
        # gradient of speed, fitted per point, then the fused LCP on it
        gout = [torch.empty((721, 1440), device="cuda") for _ in range(4)]

        def sgfit():
            P.lib().pdiv_speed_gradient_moments(
                P._p(u.data_ptr()), P._p(v.data_ptr()), 0, 50, 721, 1440, 0, 1.0, 1.0, 1,
                *[P._p(o.data_ptr()) for o in gout], 0, P._stream())

        sgfit()
        t = time_launches(sgfit, 10, torch)
        b = 2 * 50 * 721 * 1440 * 4 + 4 * 4 * 721 * 1440
        gdm, _ = P.divergence_gaussian(*gout)
        iso_g = np.quantile(gdm[::4, ::4].double().cpu().numpy(), [0.5, 0.9]).astype(np.float32)
        del gdm
        gl = torch.empty((2, 720, 1439), device="cuda")
        t2 = time_launches(lambda: (sgfit(), P.lcp_from_moments(*gout, iso_g, out=gl)), 10, torch)
        legs["speed_gradient_fit_721x1440_m50_f32"] = {
            "ms": round(t * 1e3, 4), "achieved_GBs": round(b / t / 1e9, 1),
            "frac_hbm": round(b / t / 1e9 / HBM_PEAK_GBS, 4),
            "pipeline_with_lcp_k2_ms": round(t2 * 1e3, 4)}
        del gout, gl
        c2out = torch.empty((8, 720, 1439), device="cuda")
        t = time_launches(lambda: (fit(), P.lcp_from_moments(*outs, c2["isovalues"], out=c2out)),
                          10, torch)
        legs["pipeline_fit_then_lcp_721x1440_m50_k8"] = {"ms": round(t * 1e3, 4),
                                                        "cells_per_s": round(720 * 1439 * 8 / t, 1)}
        # the error and time curve of Sec. 4 (Fig. 4): the Monte Carlo at
        # growing sample counts against the closed form on the fitted
        # ensemble; a run of S samples is the prefix of any longer run with
        # the same seed (Philox counters), and on interior cells the expected
        # SSE is sum L(1-L)/S
        iso2 = c2["isovalues"]
        P.lcp_from_moments(*outs, iso2, out=c2out)
        t_cf = time_launches(lambda: P.lcp_from_moments(*outs, iso2, out=c2out), 10, torch)
        Lh = c2out.double().cpu().numpy()
        inner = np.zeros((720, 1439), bool)
        inner[1:719, 1:1438] = True  # cells 1 <= i <= nx-3, 1 <= j <= ny-3
        var_sum = float(np.sum((Lh * (1 - Lh))[:, inner]))
        mco = torch.empty_like(c2out)
        curve = []
        for S in (10, 30, 100, 300, 1000):
            P.mc_lcp(*outs, iso2, n_samples=S, seed=2025, out=mco)
            t = time_launches(lambda: P.mc_lcp(*outs, iso2, n_samples=S, seed=2025, out=mco), 3,
                              torch)
            d2 = (mco.double().cpu().numpy() - Lh) ** 2
            curve.append({"samples": S, "ms": round(t * 1e3, 3),
                          "sse_interior": round(float(d2[:, inner].sum()), 3),
                          "expected_sse_interior": round(var_sum / S, 3),
                          "sse_all_cells": round(float(d2.sum()), 3)})
        legs["mc_error_and_time_vs_samples_721x1440_k8"] = {
            "closed_form_ms": round(t_cf * 1e3, 4), "seed": 2025, "curve": curve}
        del mco, d2
        # spaghetti plot: every member's divergence contour at the middle
        # isovalue; the binding makes one counting pdiv_spaghetti call, reads
        # the total (one host synchronisation), then the writing call
        c_sp = float(c2["isovalues"][4])
        P.spaghetti(u[:2], v[:2], c_sp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sp = P.spaghetti(u, v, c_sp)
        torch.cuda.synchronize()
        t_sp = time.perf_counter() - t0
        legs["spaghetti_721x1440_m50"] = {"ms": round(t_sp * 1e3, 3),
                                          "segments": int(sum(int(x.shape[0]) for x in sp))}
        del sp
        del u, v, outs, c2out
        torch.cuda.empty_cache()
        legs["batch_512_fields_k4"] = guarded("batch leg", batch_leg, P, synth, torch, np)
        torch.cuda.empty_cache()
        legs["volume_3d_512"] = guarded("3D leg", volume_leg, P, synth, torch, np)
        torch.cuda.empty_cache()
        legs["served_stream"] = guarded("served leg", served_leg, P, synth, torch, np)
        result["legs"] = legs

    if not args.no_cpu_baseline:
        import oracle as O

        rows = (2048, 6144)
        log(f"CPU baseline: FP64 oracle on cell rows {rows[0]}..{rows[1]} (1 thread)")
        stored = [t.double().cpu().numpy() for t in mom]
        t_cpu = 0.0
        n_cpu = 0
        worst = 0.0
        sum_err = 0.0
        # LCP bins of the oracle value (add_to_bins)
        bins = new_bins()
        for j0 in range(rows[0], rows[1], 256):
            j1 = min(j0 + 256, rows[1])
            a, b = j0 - 1, j1 + 2
            t = time.perf_counter()
            m, vv = O.divergence_gaussian(*[x[a:b] for x in stored], 1.0, 1.0)
            ref = O.lcp(m[1:-1], vv[1:-1], iso)
            t_cpu += time.perf_counter() - t
            n_cpu += ref.size
            g = out[:, j0:j1, :].double().cpu().numpy()
            err = np.abs(g - ref)
            worst = max(worst, float(np.max(err)))
            sum_err += float(err.sum())
            add_to_bins(bins, ref, err, np)
        cpu = n_cpu / t_cpu
        result["cpu_baseline"] = {"value": round(cpu, 1), "unit": "LCP cells/s",
                                  "cores": 1, "kind": "oracle",
                                  "sample": f"cell rows {rows[0]}-{rows[1] - 1} of the same "
                                            f"8192x8192 field, all {K} isovalues "
                                            f"({n_cpu} LCP values, {t_cpu:.1f} s, numpy float64)",
                                  "gpu_speedup": round(value / cpu, 1),
                                  "gpu_max_abs_err_on_sample": worst,
                                  "host": host_cpu()}
        if not args.no_cpu_legs:
            legs_cpu = guarded("CPU legs", cpu_legs, stored, iso, rows, mc_target=args.mc_samples)
            result["cpu_baseline"].update(legs_cpu if "error" not in legs_cpu
                                          else {"cpu_legs_error": legs_cpu["error"]})
        if not args.no_cpu_legs and "error" not in legs_cpu:
            mc1 = legs_cpu["mc_1core"]["value"]
            ratios = {"cpu_oracle_1core_vs_cpu_mc_1core": round(cpu / mc1, 1),
                      "cpu_oracle_all_cores_vs_cpu_mc_1core":
                          round(legs_cpu["oracle_all_cores"]["value"] / mc1, 1),
                      "gpu_closed_form_vs_cpu_mc_1core": round(value / mc1, 1)}
            if "mc" in result:
                ratios["gpu_closed_form_vs_gpu_mc"] = result["mc"]["closed_form_speedup"]
            # the paper's speed-ups of the closed form over serial Monte Carlo,
            # on its own hardware and datasets (Sec. 4): context only
            ratios["paper_context"] = {
                "wind_serial_closed_form_vs_serial_mc": 1946,
                "wind_openmp10_closed_form_vs_serial_mc": 9891,
                "red_sea_serial_closed_form_vs_serial_mc": 1125.62,
                "red_sea_openmp10_closed_form_vs_serial_mc": 10505.8,
                "red_sea_gpu_closed_form_vs_serial_mc": 19698.37,
                "hardware": "Apple M4 (serial and 10 threads); a GPU of the Frontier system"}
            result["cpu_baseline"]["ratios"] = ratios
        result["accuracy"] = {"max_abs_err_vs_fp64_oracle": worst, "bar": 1e-5,
                              "within_bar": worst <= 1e-5,
                              "mean_abs_err_vs_fp64_oracle": sum_err / n_cpu,
                              "sample": f"cell rows {rows[0]}-{rows[1] - 1}, float32 storage, "
                                        "oracle on the stored values",
                              "bins_by_oracle_lcp": bins}
        # storage precision: every storage type on one band, against the
        # oracle on its stored values (kernel arithmetic) and on the float64
        # field (end to end, storage rounding included)
        a0, a1 = 4096, 4352
        keys = ("mean_u", "var_u", "mean_v", "var_v")
        m64, v64 = O.divergence_gaussian(*[c3[k][a0 - 1:a1 + 2] for k in keys], 1.0, 1.0)
        ref_e2e = O.lcp(m64[1:-1], v64[1:-1], iso)
        prec = {"sample": f"cell rows {a0}-{a1 - 1}, all {K} isovalues"}
        for name, dt in (("f32", torch.float32), ("f16", torch.float16),
                         ("bf16", torch.bfloat16)):
            ts = [torch.from_numpy(c3[k]).to(dt).cuda() for k in keys]
            g = P.lcp_from_moments(*ts, iso)[:, a0:a1, :].double().cpu().numpy()
            st = [t[a0 - 1:a1 + 2].double().cpu().numpy() for t in ts]
            del ts
            ms, vs = O.divergence_gaussian(*st, 1.0, 1.0)
            e_k = np.abs(g - O.lcp(ms[1:-1], vs[1:-1], iso))
            e_e = np.abs(g - ref_e2e)
            prec[name] = {"kernel_max_abs": float(e_k.max()), "kernel_mean_abs": float(e_k.mean()),
                          "end_to_end_max_abs": float(e_e.max()),
                          "end_to_end_mean_abs": float(e_e.mean())}
        torch.cuda.empty_cache()
        result["accuracy"]["storage_precision"] = prec
        del c3
        result["accuracy"]["near_0_1_low_spread"] = guarded("near-0/1 leg", near01_leg, P,
                                                            synth, torch, np)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
