"""Host logic of bench.py (no GPU): the one-GPU contract, the default line
and its time plan, and the guard that ties a committed HBM-traffic figure
to the kernel sources it was measured on."""
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


def test_default_line_is_the_batched_gate_workload():
    a = bench.parse([])
    assert (a.workload, a.steps, a.warmup, a.chains) == ("gate", 20, 5, None)
    assert a.precision == "fp64" and not a.no_extras
    assert bench.DEFAULT_CHAINS == 64
    assert workloads.M1.chi == 256 and workloads.M1.chi_max == 256
    a = bench.parse(["--workload", "m1", "--steps", "3", "--warmup", "0"])
    assert (a.steps, a.warmup) == (3, 0)


def test_the_drivers_command_fits_its_time_limit():
    # the full test run is `bench.py --gpus 1 --steps 20 --warmup 5` under a
    # 600 s limit; its planned work at half the measured rates (first torch
    # import on a fresh box included) must leave a wide margin
    a = bench.parse(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert bench.planned_seconds(a) < 400
    assert bench.planned_seconds(bench.parse([])) < 400
    # whole ladder samples are minutes per step: never the default
    assert bench.planned_seconds(bench.parse(["--workload", "c3"])) == \
        float("inf")


def test_traffic_is_used_only_for_the_measured_sources(monkeypatch):
    found = []
    for f in os.listdir(os.path.join(ROOT, "profiles")):
        if "_traffic_" in f and f.endswith(".md"):
            kernel, tag = f[:-3].split("_traffic_", 1)
            found.append((kernel, tag, f))
    for kernel, tag, f in found:
        t = bench.measured_traffic(kernel, tag)
        recorded = None
        with open(os.path.join(ROOT, "profiles", f)) as fh:
            for line in fh:
                if line.startswith("source_sha256:"):
                    recorded = line.split(":", 1)[1].strip().strip("`")
        if recorded == bench.kernel_source_hash():
            assert t is not None and t > 0
        else:
            assert t is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    for kernel, tag, _ in found:
        assert bench.measured_traffic(kernel, tag) is None
    # a workload without a counter summary has no traffic figure
    assert bench.measured_traffic("k_jacobi_round", workloads.C1.name) is None
    assert bench.measured_traffic("k_jacobi_round_wide",
                                  workloads.C1.name) is None


def test_oracle_baseline_on_a_small_bond():
    # the oracle leg of the gate workload on a reduced bond (chi 12)
    wl = workloads.BondWorkload("bond_chi12", 12, 1.0, 0.025, 12, 1e-10,
                                24.0)
    center, right = workloads.bond_tensors(0, 1, 12, 12, 12)
    cb = bench.cpu_baseline_bond(wl, center, right, 0.06)
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    assert cb["single_core_value"] > 0
    assert "gate applications" in cb["sample"]
    for key in ("cpu_model", "blas", "blas_threads", "os_cpu_count"):
        assert key in cb


def test_charge_histogram():
    # integer <Q> (S^z environments) counted per value, the rest apart
    h = bench.qn_histogram([0.0, 1.0 + 1e-9, -2.0, 0.5, 1.0, -2.0])
    assert h == {"-2": 2, "0": 1, "1": 2, "not_integer": 1}
    assert list(h)[:3] == ["-2", "0", "1"]
