"""The serving policy (admission by HBM budget, LRU eviction of fields no
request names, merging of slider requests into one launch per free slot,
failure isolation, memory and latency bookkeeping) against a fake executor
and a virtual clock.  The policy is the header the server library compiles;
the driver is host C++ built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer.  CPU only."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host_checks", "server_core_test.cpp")


def test_server_policy_with_fake_executor(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "server_core_test")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ALL PASS" in r.stdout
    for name in ("upload_then_sliders_merge", "one_launch_per_free_slot",
                 "lru_eviction_skips_referenced", "fifo_admission_blocks_later_fields",
                 "failed_upload_isolated", "failed_launch_isolated", "shutdown_fails_queued",
                 "dtype_staging_bytes", "random_soak"):
        assert f"PASS {name}" in r.stdout


def test_monte_carlo_rank_table(tmp_path):
    """The Monte Carlo kernel's sorted isovalue table (csrc/mc_rank.hpp):
    the search the kernel takes gives every value's rank over the chunk,
    with ties, infinities, empty slots, 8 and 16 slots; NaN isovalues are
    refused.  Host C++ under AddressSanitizer and UndefinedBehaviorSanitizer."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "mc_rank_test")
    src = os.path.join(HERE, "host_checks", "mc_rank_test.cpp")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ALL PASS" in r.stdout
