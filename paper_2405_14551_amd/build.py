"""Build the HIP library ``liblbmi.so`` in-tree for gfx950.

Every ``csrc/*.hip`` file is compiled to an object in ``_build/`` (in
parallel) and the objects are linked into ``paper_2405_14551_amd/liblbmi.so``.
Run ``python -m paper_2405_14551_amd.build`` or call ``build()``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
# LB_BUILD_DIR / LB_LIB_OUT: another object directory and library path (for
# builds with other compile-time settings, LB_EXTRA_CFLAGS, e.g. -DLB_RO_PIPELINE=0)
BUILD = os.environ.get("LB_BUILD_DIR", os.path.join(ROOT, "_build"))
LIB = os.environ.get("LB_LIB_OUT", os.path.join(PKG, "liblbmi.so"))
ARCH = os.environ.get("LB_OFFLOAD_ARCH", "gfx950")
EXTRA = os.environ.get("LB_EXTRA_CFLAGS", "").split()

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-fPIC",
    "-std=c++17",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
    "-Wno-unused-lambda-capture",
    # no packed FP32 instructions in generated device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    *EXTRA,
]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    # the heaviest translation units (D3Q27, then D3Q19 collision passes) first,
    # so that the parallel build does not end on one long compile
    def cost(path):
        name = os.path.basename(path)
        lat = 0 if "d3q27" in name else (1 if "d3q19" in name else 2)
        return (lat, 0 if "collide" in name else 1, name)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")), key=cost)
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
