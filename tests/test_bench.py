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


def test_step_defaults_follow_the_workload(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert (a.workload, a.steps, a.warmup) == ("c3", 1, 0)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "m1"])
    a = bench.parse()
    assert (a.steps, a.warmup) == (20, 2)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "m1",
                                      "--steps", "3", "--warmup", "0"])
    a = bench.parse()
    assert (a.steps, a.warmup) == (3, 0)


def test_gate_workload_has_no_traffic_figure():
    # the committed counters cover the ladder workload only
    assert bench.measured_traffic(workloads.M1) is None


def test_oracle_baseline_on_a_small_bond():
    # the oracle leg of the gate workload on a reduced bond (chi 12)
    wl = workloads.BondWorkload("bond_chi12", 12, 1.0, 0.025, 12, 1e-10,
                                24.0)
    center, right = workloads.bond_tensors(0, 1, 12, 12, 12)
    cb = bench.cpu_baseline_bond(wl, center, right, 0.05)
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    assert "gate applications" in cb["sample"]
