"""Builds libpdiv.so (gfx950) in-tree with hipcc.

Every library source under csrc/ is compiled for gfx950 with packed-FP32
code generation switched off, then linked into paper_2510_01190_amd/libpdiv.so.
csrc/probe_valu_costs.hip, a standalone measuring program (not linked into
the library), is built next to it as paper_2510_01190_amd/probe_valu_costs.
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
PROBE_SRC = "probe_valu_costs.hip"
PROBE = os.path.join(HERE, "probe_valu_costs")

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


# Host-side sanitizers for the checking build: AddressSanitizer and
# UndefinedBehaviorSanitizer on the host code only (each flag after
# -Xarch_host); the device code is compiled as usual.
SANITIZE_FLAGS = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                  "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """Path of clang's shared AddressSanitizer runtime, which a process
    loading the sanitized library must preload."""
    import glob
    root = os.path.join(os.path.dirname(os.path.dirname(_hipcc())), "lib", "llvm", "lib",
                        "clang")
    hits = sorted(glob.glob(os.path.join(root, "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("clang's AddressSanitizer runtime not found")
    return hits[-1]


def build(verbose: bool = False, jobs: int | None = None, sanitize: bool = False,
          out_dir: str | None = None) -> str:
    """Compiles every source (always, even if a library exists) and links
    libpdiv.so.  sanitize=True builds the host-sanitized variant
    (libpdiv_san.so, in out_dir), for checking runs only."""
    hipcc = _hipcc()
    obj_dir = os.path.join(out_dir, "obj") if out_dir else OUT
    os.makedirs(obj_dir, exist_ok=True)
    flags = CFLAGS + SANITIZE_FLAGS if sanitize else CFLAGS
    lib_path = os.path.join(out_dir, "libpdiv_san.so" if sanitize else "libpdiv.so") \
        if out_dir else LIB

    def compile_one(src: str) -> str:
        obj = os.path.join(obj_dir, src.rsplit(".", 1)[0] + ".o")
        cmd = [hipcc, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=jobs or min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = lib_path + ".tmp"
    link = ["-fsanitize=address,undefined", "-shared-libasan"] if sanitize else []
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *link, "-o", tmp, *objs,
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib_path)
    if not sanitize and not out_dir:
        build_probe(hipcc)
    return lib_path


def build_probe(hipcc: str | None = None) -> str:
    """Compiles the vector-ALU issue-cost probe (an executable)."""
    hipcc = hipcc or _hipcc()
    tmp = PROBE + ".tmp"
    cmd = [hipcc, *[f for f in CFLAGS if f not in ("-fPIC", "-munsafe-fp-atomics")],
           os.path.join(CSRC, PROBE_SRC), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {PROBE_SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, PROBE)
    return PROBE


if __name__ == "__main__":
    print(build(verbose=True))
