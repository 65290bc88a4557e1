"""Host logic of bench.py (no GPU): the single-GPU guard and the lookup of
counted HBM traffic, which must only be reported for the kernel source and
tile shape it was measured on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus 2 is not supported" in r.stderr
    assert r.stdout == ""


def test_traffic_lookup_needs_matching_source_and_tile(tmp_path, monkeypatch):
    path = tmp_path / "traffic.json"
    entry = {"tile": [5, 256, 2, 7], "bytes_per_pass_launch": 123456789.0}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic([5, 256, 2, 7]) is None  # no file
    path.write_text(json.dumps({"kernel_sha256_16": bench.kernel_hash(), "entries": [entry]}))
    assert bench.measured_traffic([5, 256, 2, 7]) == 123456789.0
    assert bench.measured_traffic([5, 256, 2, 6]) is None  # another tile
    path.write_text(json.dumps({"kernel_sha256_16": "0" * 16, "entries": [entry]}))
    assert bench.measured_traffic([5, 256, 2, 7]) is None  # another kernel source
    path.write_text("not json")
    assert bench.measured_traffic([5, 256, 2, 7]) is None


def test_kernel_hash_covers_every_device_source():
    from paper_2106_11286_amd import build as B

    files = B.kernel_source_files()
    names = {os.path.basename(f) for f in files}
    for src in B.KERNEL_SOURCES:
        assert src in names
    assert "device_common.hpp" in names and "build.py" in names
    assert len(bench.kernel_hash()) == 16
