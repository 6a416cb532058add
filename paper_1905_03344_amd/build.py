"""Build libsph.so (HIP kernels for gfx950 + the C ABI host layer) in-tree.

    python -m paper_1905_03344_amd.build [-v]

Every .hip source is compiled for gfx950 only.  Packed FP32 instructions
are disabled (`-target-feature -packed-fp32-ops`).  Contraction follows the
per-function `#pragma clang fp contract(off)` of the exact neighbour-test and
integrator code; field kernels may contract.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libsph.so")
BUILD = os.path.join(HERE, "_build")

HIP_SOURCES = ["cells.hip", "neighbors.hip", "physics.hip", "mixed.hip", "mlp.hip"]
CXX_SOURCES = ["api.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-I", INCLUDE, "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable"]
HIP_FLAGS = ["--offload-arch=gfx950", "-ffp-contract=fast-honor-pragmas", "-Xclang",
             "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _compile(src: str, verbose: bool) -> str:
    os.makedirs(BUILD, exist_ok=True)
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    if src.endswith(".hip"):
        cmd = [_hipcc(), "-x", "hip", *HIP_FLAGS, *COMMON, "-c", path, "-o", obj]
    else:
        cmd = [_hipcc(), "--offload-arch=gfx950", *COMMON, "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    srcs = [s for s in HIP_SOURCES + CXX_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
