"""Host logic of bench.py (no GPU): the one-GPU contract and the guard
that ties a committed HBM-traffic figure to the kernel sources it was
measured on."""
import os
import subprocess
import sys

import bench
from paper_1910_09142_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_used_only_for_the_measured_sources(monkeypatch):
    t = bench.measured_traffic(workloads.C3)
    path = os.path.join(ROOT, "profiles",
                        f"k_jacobi_round_traffic_{workloads.C3.name}.md")
    recorded = None
    with open(path) as f:
        for line in f:
            if line.startswith("source_sha256:"):
                recorded = line.split(":", 1)[1].strip().strip("`")
    if recorded == bench.kernel_source_hash():
        assert t is not None and t > 0
    else:
        assert t is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic(workloads.C3) is None
    # a workload without a counter summary has no traffic figure
    assert bench.measured_traffic(workloads.C1) is None


def test_prefix_rate_covers_the_oracle_updates():
    marks = [(i, 100.0 + 2.0 * i) for i in range(1, 51)]
    # 2573 updates at 252 per Trotter step need 11 steps
    assert bench.prefix_rate(marks, 100.0, 2573, 252.0) == (11, 2772, 126.0)
    assert bench.prefix_rate(marks, 100.0, 252, 252.0) == (1, 252, 126.0)
    assert bench.prefix_rate([], 100.0, 10, 252.0) is None
    assert bench.prefix_rate(marks, 100.0, 10 ** 9, 252.0) is None
    assert bench.model_steps(workloads.C3) == 50
