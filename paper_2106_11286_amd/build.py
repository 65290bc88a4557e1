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
# device code: one translation unit per launch family (compiled in parallel)
KERNEL_SOURCES = ["kernels_pass.hip", "kernels_basis_pair.hip", "kernels_persistent.hip",
                  "kernels_lds.hip", "kernels_util.hip", "kernels_block.hip",
                  "kernels_measure.hip", "kernels_fused.hip"]
# host runtime behind the C ABI
HOST_SOURCES = ["abi.cpp", "abi_tune.cpp", "abi_stats.cpp", "abi_extensions.cpp"]
# host entry point that shares its translation unit with a static device array
MIXED_SOURCES = ["abi_noalloc.hip"]
SOURCES = KERNEL_SOURCES + HOST_SOURCES + MIXED_SOURCES
ARCH = os.environ.get("MCHEIS_ARCH", "gfx950")


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return p


def compile_flags():
    """(host-and-device flags, device flags) used for every source."""
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
    return common, dev


def kernel_source_files():
    """Every file the device code is compiled from, plus this build script."""
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp")))
    return [os.path.join(CSRC, f) for f in names] + [os.path.abspath(__file__)]


def build(verbose: bool = False) -> str:
    """Compile every source into ``libmcheis.so`` (always recompiles)."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common, dev = compile_flags()

    def compile_one(src):
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc()] + common + dev + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    workers = max(1, min(len(SOURCES), os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
