"""Builds libpdiv.so (gfx950) in-tree with hipcc.

Every source under csrc/ is compiled for gfx950 with packed-FP32 code
generation switched off, then linked into paper_2510_01190_amd/libpdiv.so.
Run as `python -m paper_2510_01190_amd.build_lib` or through build().
"""

from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpdiv.so")

SOURCES = ["pdiv_api.hip", "k_moments.hip", "k_lcp.hip", "k_lcp3d.hip", "k_speed_gradient.hip",
           "k_contour.hip", "k_mc.hip", "pdiv_batch.hip", "pdiv_server.hip"]

ARCH = "gfx950"
CFLAGS = [f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found: cannot build libpdiv")
    return h


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compiles every source (always, even if a library exists) and links libpdiv.so."""
    hipcc = _hipcc()
    os.makedirs(OUT, exist_ok=True)

    def compile_one(src: str) -> str:
        obj = os.path.join(OUT, src.rsplit(".", 1)[0] + ".o")
        cmd = [hipcc, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=jobs or min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
