"""The input generator checks itself against its closed form, and the bench
refuses more than one GPU.  CPU only."""

import os
import subprocess
import sys

import numpy as np

import oracle as O
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_generator_divergence_is_second_order_consistent():
    """Interior central differences of the generated mean field approach the
    generator's analytic divergence as O(h^2): halving the feature scale
    relative to the grid (doubling widths) cuts the error about fourfold."""
    errs = []
    for scale in (1.0, 2.0):
        feats = [synth.Feature(80.0, 80.0, 1.5, 8.0 * scale, False)]  # one source
        u, v = synth.mean_field(feats, 160, 160)
        d = synth.analytic_divergence(feats, 160, 160)
        fd = O.fd_divergence(u, v, 1.0, 1.0)
        errs.append(np.max(np.abs(fd - d)[2:-2, 2:-2]) * scale)  # relative to the peak A/w
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_vortex_has_zero_divergence():
    feats = [synth.Feature(40.0, 50.0, 1.0, 10.0, True)]
    u, v = synth.mean_field(feats, 100, 90)
    assert np.all(synth.analytic_divergence(feats, 100, 90) == 0.0)
    fd = O.fd_divergence(u, v, 1.0, 1.0)
    assert np.max(np.abs(fd[2:-2, 2:-2])) < 1e-3


def test_configs_are_seeded_and_shaped():
    a, b = synth.config_c1(), synth.config_c1()
    assert np.array_equal(a["mean_u"], b["mean_u"]) and a["mean_u"].shape == (128, 128)
    assert a["isovalues"].dtype == np.float32 and a["n_samples"] == 2000
    s = synth.batch_sizes(512, 64, 2048, synth.SEED_BASE + 4)
    sides = np.array(s)
    assert sides.min() >= 64 and sides.max() <= 2048 and len(s) == 512


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
