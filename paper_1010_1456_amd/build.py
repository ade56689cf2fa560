"""Builds libaim.so (HIP for gfx950) in-tree.

    python -m paper_1010_1456_amd.build

Every source is compiled with hipcc for gfx950 only. The host planner is
compiled with -ffp-contract=off so that its floating-point decisions (stencil
anchors, near-zone distances) are free of fused multiply-adds. Packed FP32
instructions are disabled on the device side.
"""

from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libaim.so")
BUILD = os.path.join(HERE, "_build")
ARCH = "gfx950"

SOURCES = ["host_plan.cpp", "api.hip", "setup_kernels.hip", "matvec.hip", "solver.hip", "rcs.hip",
           "fft_contig_f32.hip", "fft_contig_f64.hip", "fft_strided_f32.hip", "fft_strided_f64.hip",
           "fft_mid_f32.hip", "fft_mid_f64.hip", "fft_anterp_f32.hip", "fft_anterp_f64.hip",
           "fft_xy_f32.hip", "fft_xy_f64.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
          "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    args = [hipcc(), *COMMON, "-c", os.path.join(SRC, src), "-o", obj]
    if src.endswith(".cpp"):
        args[1:1] = ["-x", "hip", "-ffp-contract=off"]
    else:
        args[1:1] = ["-x", "hip"]
    r = subprocess.run(args, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(max(os.cpu_count() or 8, 1), 16, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    args = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(args, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
