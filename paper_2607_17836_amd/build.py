"""Build liblpt.so and libns2d.so (gfx950) in-tree with hipcc.

    python -m paper_2607_17836_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblpt.so")
SOURCES = ["runtime.cpp", "step.hip", "sort.hip", "probe.hip", "adjoint.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # code object v5 loads under both the ROCm 7.0 runtime bundled with torch
    # and the system ROCm 7.2 runtime
    "-mcode-object-version=5",
    # packed-FP32 instructions stay off: plain scalar/float2 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function",
]


NS_LIB = os.path.join(PKG, "libns2d.so")
NS_SOURCES = [os.path.join(PKG, "csrc_ns", "ns2d.hip")]
ROCM_LIB = "/opt/rocm/lib"


def build_ns(verbose: bool = False) -> str:
    """libns2d.so: the Eulerian field producer (hipFFT transforms)."""
    tmp = NS_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), *NS_SOURCES,
           "-L", ROCM_LIB, "-lhipfft", "-Wl,-rpath," + ROCM_LIB, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, NS_LIB)
    return NS_LIB


def build(verbose: bool = False) -> str:
    build_ns(verbose)
    srcs = []
    for s in SOURCES:
        path = os.path.join(CSRC, s)
        # .cpp host sources go through hipcc as HIP too (they use the HIP runtime)
        srcs += (["-x", "hip", path] if s.endswith(".cpp") else [path])
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
