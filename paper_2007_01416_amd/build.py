"""Build the gfx950 HIP library in-tree: paper_2007_01416_amd/libacat.so.

    python -m paper_2007_01416_amd.build

Every translation unit is compiled with hipcc for gfx950 only, with packed
fp32 instruction selection disabled, and linked into one shared library with
a plain C ABI (include/acat.h).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libacat.so")
SOURCES = ["acat_step.hip", "acat_batched.hip", "acat_adjoint.hip", "acat_api.hip", "acat_measure.hip",
           "acat_profile.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -ffp-contract=off: no implicit fused multiply-add; the forward kernels
# write every fma they use explicitly, so the rounding of each operation is
# fixed (the adjoint's translation unit is the exception, CONTRACT below).
# -fconstexpr-steps: the coefficient tables (exact rationals up to 12 nodes)
# are evaluated at compile time.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=off",
         "-fconstexpr-steps=400000000",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


# The adjoint is checked against the oracle at a tolerance, not bit for bit:
# its products and sums may be fused by the compiler.
CONTRACT = {"acat_adjoint.hip": "-ffp-contract=fast"}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    flags = [CONTRACT.get(src, f) if f == "-ffp-contract=off" else f for f in FLAGS]
    cmd = [HIPCC, *flags, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
