"""Host logic of the benchmark script (no GPU): the one-GPU guard and the
gating of the measured HBM traffic by kernel source and configuration."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_reported_only_for_the_measured_source_and_groups():
    for (family, streams), m in bench.MEASURED_TRAFFIC.items():
        same = True
        for src, sha in m["sources"].items():
            with open(os.path.join(ROOT, src), "rb") as f:
                same = same and hashlib.sha256(f.read()).hexdigest() == sha
        assert bench.measured_traffic(family, streams) == (m["bytes_per_launch"] if same else None)
        assert bench.measured_traffic(family, streams + 1) is None
    assert bench.measured_traffic("jacobi", 3) is None
