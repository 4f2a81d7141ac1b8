"""Host logic of bench.py (no GPU): the source files whose hash keys the
measured HBM traffic, the staleness rule for that traffic, and the one-GPU
guard of the command line."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("kernel", sorted(bench.KERNEL_ROOTS))
def test_kernel_sources_are_the_include_closure(kernel):
    files = bench.kernel_sources(kernel)
    assert files[0] == bench.KERNEL_ROOTS[kernel]
    assert len(set(files)) == len(files)
    assert "paper_1009_3308_amd/csrc/nse_internal.h" in files
    assert "include/nse_sphere.h" in files
    # closed: every local include of every listed file is listed
    names = {os.path.basename(f) for f in files}
    for f in files:
        with open(os.path.join(ROOT, f)) as fh:
            for inc in re.findall(r'^\s*#\s*include\s+"([^"]+)"', fh.read(), re.M):
                assert os.path.basename(inc) in names, (f, inc)


def test_synthesis_and_analysis_hash_their_device_headers():
    for kernel in ("synthesis", "analysis"):
        names = {os.path.basename(f) for f in bench.kernel_sources(kernel)}
        assert {"lane_ops.h", "spectral_ops.h", "ndf_device.h", "ndf_control.h"} <= names


def test_traffic_is_reported_only_for_unchanged_sources(tmp_path, monkeypatch):
    workload = "some workload"
    entries = [
        {"kernel": "ring", "workload": workload, "bytes_per_launch": 123,
         "source_sha256": bench.source_sha("ring")},
        {"kernel": "analysis", "workload": workload, "bytes_per_launch": 456,
         "source_sha256": "0" * 64},
    ]
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(entries))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic("ring", workload) == 123
    assert bench.measured_traffic("analysis", workload) is None  # stale hash
    assert bench.measured_traffic("ring", "another workload") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("ring", workload) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
