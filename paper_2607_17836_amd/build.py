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


def _compile(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.run(cmd).returncode


def build(verbose: bool = False) -> str:
    """Compile every source of liblpt.so to an object (in parallel), link the
    library in-tree, then build libns2d.so."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(ROOT, "_build", "lpt")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for s in SOURCES:
        path = os.path.join(CSRC, s)
        obj = os.path.join(objdir, s + ".o")
        # .cpp host sources go through hipcc as HIP too (they use the HIP runtime)
        src = ["-x", "hip", path] if s.endswith(".cpp") else [path]
        flags = [f for f in FLAGS if f != "-shared"]
        cmds.append([HIPCC, *flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", *src,
                     "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=min(len(cmds) + 1, os.cpu_count() or 4)) as ex:
        ns = ex.submit(build_ns, verbose)
        codes = list(ex.map(lambda c: _compile(c, verbose), cmds))
        ns.result()
    if any(codes):
        raise subprocess.CalledProcessError(max(codes), "hipcc (liblpt.so objects)")
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
