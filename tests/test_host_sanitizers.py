"""The library's host code (argument checks, batch and server bookkeeping)
under AddressSanitizer and UndefinedBehaviorSanitizer: a host-sanitized
build runs every C-ABI check of test_abi.py in a child process that preloads
the sanitizer runtime; any report aborts it.  CPU only: the calls the ABI
tests make are rejected before any device work."""

import os
import subprocess
import sys

import pytest

from paper_2510_01190_amd import build_lib

HERE = os.path.dirname(os.path.abspath(__file__))

pytestmark = pytest.mark.slow


def test_abi_checks_are_clean_under_asan_and_ubsan(tmp_path):
    try:
        runtime = build_lib.asan_runtime()
        lib = build_lib.build(sanitize=True, out_dir=str(tmp_path))
    except RuntimeError as e:
        pytest.skip(f"no sanitizer build here: {e}")
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:print_summary=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, os.path.join(HERE, "host_checks", "run_abi_tests.py"), lib],
                       env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout
