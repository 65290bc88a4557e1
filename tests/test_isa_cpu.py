"""Static checks of the generated gfx950 code (CPU only: compiles the kernel
source to assembly).  Stores and atomics must go through vector memory: the
scalar data cache is never written, and no kernel spills to scratch."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2106_11286_amd", "csrc")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("isa") / "kernels.s")
    subprocess.check_call([hipcc, "-std=c++17", "-O3", "-x", "hip", "--offload-arch=gfx950",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-fgpu-flush-denormals-to-zero", "-I", os.path.join(ROOT, "include"),
                           "-I", CSRC, "--offload-device-only", "-S", "-o", out,
                           os.path.join(CSRC, "kernels.hip")], stderr=subprocess.DEVNULL)
    return open(out).read()


def test_no_scalar_memory_writes(asm):
    bad = re.compile(r"^\s*(s_store_|s_buffer_store|s_scratch_store|s_atomic_|s_buffer_atomic|"
                     r"s_dcache_wb|s_dcache_discard)", re.M)
    hits = bad.findall(asm)
    assert not hits, sorted(set(hits))


def test_no_scratch_spills(asm):
    spills = [int(v) for v in re.findall(r"\.vgpr_spill_count:\s+(\d+)", asm)]
    assert spills and max(spills) == 0
    for m in re.finditer(r"\.private_segment_fixed_size:\s+(\d+)", asm):
        assert int(m.group(1)) == 0
