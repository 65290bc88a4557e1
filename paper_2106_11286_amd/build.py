"""Build the HIP library ``libmcheis.so`` in-tree for gfx950 (MI355X).

Usage: ``python -m paper_2106_11286_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmcheis.so")
SOURCES = ["kernels.hip", "abi.cpp"]
ARCH = os.environ.get("MCHEIS_ARCH", "gfx950")


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return p


def build(verbose: bool = False) -> str:
    """Compile every source into ``libmcheis.so`` (always recompiles)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["-std=c++17", "-O3", "-fPIC", "-I", INCLUDE, "-I", CSRC,
              "-Wall", "-Wno-unused-function"]
    dev = ["-x", "hip", "--offload-arch=" + ARCH,
           # packed FP32 ops are kept out of the generated code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-fgpu-flush-denormals-to-zero",
           # multiply-adds fuse only within one source expression, so every
           # instantiation of a pass body (measured or not, any tile shape)
           # rounds the same way and the Markov chain does not depend on it
           "-ffp-contract=on"]
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc()] + common + dev + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
