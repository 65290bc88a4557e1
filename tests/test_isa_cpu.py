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
    """Assembly of every device source, compiled with the library's own flags."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    import sys

    sys.path.insert(0, ROOT)
    from concurrent.futures import ThreadPoolExecutor

    from paper_2106_11286_amd import build as B

    common, dev = B.compile_flags()
    d = tmp_path_factory.mktemp("isa")

    def one(src):
        out = str(d / (src + ".s"))
        subprocess.check_call([hipcc] + common + dev + ["--offload-device-only", "-S", "-o", out,
                                                        os.path.join(CSRC, src)],
                              stderr=subprocess.DEVNULL)
        return open(out).read()

    with ThreadPoolExecutor(max_workers=len(B.KERNEL_SOURCES)) as pool:
        return "\n".join(pool.map(one, B.KERNEL_SOURCES))


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
