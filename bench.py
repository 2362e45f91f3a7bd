#!/usr/bin/env python3
"""Benchmark of the hybrid METTS-ancilla hot path on one MI355X.

One step = one full sample of every chain of the batch: imaginary-time
evolution to beta/2 (every Trotter gate and swap with its truncated SVD),
measurement of every bond, projective collapse of the environment and
re-initialisation (Markov chain steps 2-4 of Chen & Stoudenmire,
arXiv:1910.09142).  The default workload is the 2x16 S=1 ladder with
J_rung = 0.5, W = 2, beta = 5, tau = 0.05, chi_max = 256, cutoff 1e-10 in
FP64 (one chain); inputs are synthetic (Philox product states).

Prints one JSON line.  `value` counts the two-site Trotter updates (gates
and swaps; orthogonality-centre moves excluded) per second of the timed
region, all chains together.

`--workload m1` measures single gate applications at chi = 256 instead:
every chain holds one bond with chi_l = chi_m = chi_r = 256 (synthetic
Haar factors, Schmidt values exp(-j/24)); one step applies exp(-(tau/2) J
S.S) with tau = 0.05, J = 1 to every chain, with the truncated SVD back to
chi_max = 256 at cutoff 1e-10, sweeping the bond back and forth.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("two-site gate apps/sec at χ=256 (FP64 vs mixed, batched); "
          "METTS samples/sec")
UNIT = "two-site gate applications/s"
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 1 sample; m1: 20 gates)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default 0; m1: 2)")
    ap.add_argument("--workload", default="c3",
                    choices=["c1", "c2", "c3", "c4", "c5", "m1"])
    ap.add_argument("--chains", type=int, default=None,
                    help="override the number of chains of the workload")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="mixed: FP32 theta contraction and gate on the "
                    "matrix cores, FP64 SVD, truncation and observables")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget of the oracle baseline (0 disables it)")
    args = ap.parse_args()
    bond = args.workload == "m1"
    if args.steps is None:
        args.steps = 20 if bond else 1
    if args.warmup is None:
        args.warmup = 2 if bond else 0
    return args


# Sources that make up the round kernel; a traffic figure measured with
# hardware counters holds only for the code it was measured on.
KERNEL_SOURCES = ("jacobi.hip", "device_common.h", "hmps_internal.h")


def kernel_source_hash():
    """SHA-256 of the round-kernel sources with comments removed and runs of
    whitespace collapsed: edits to comments keep a measurement valid, any
    change to the code does not."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1910_09142_amd", "csrc", name),
                  encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        text = " ".join(text.split())
        h.update(name.encode() + b"\0" + text.encode() + b"\0")
    return h.hexdigest()


def measured_traffic(wl):
    """HBM bytes per round-kernel launch from the committed rocprofv3
    counter summary of this workload (FETCH_SIZE and WRITE_SIZE scaled by
    the copy-kernel calibration), or None when there is none or it was
    taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles",
                        f"k_jacobi_round_traffic_{wl.name}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.split(":", 1)[0].strip() in (
                    "source_sha256", "traffic_bytes_per_launch"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def model_steps(wl):
    """Trotter steps of one evolution to beta/2."""
    return int(round(wl.beta / (2.0 * wl.tau)))


def prefix_rate(marks, t0, n_updates, per_step):
    """(steps, updates, updates/s) of the GPU over the fewest leading
    Trotter steps of the timed sample that cover n_updates, from the
    (steps done, time) marks of the progress callback; None without marks."""
    if not marks or per_step <= 0:
        return None
    need = max(1, int(-(-n_updates // per_step)))
    for done, t in marks:
        if done >= need and t > t0:
            ups = int(round(done * per_step))
            return done, ups, ups / (t - t0)
    return None


def cpu_baseline(wl, seconds):
    """The FP64 oracle on the same workload: chain 0, seed 0, sample 0,
    Trotter updates in order until the time budget is spent."""
    from oracle import model, mps
    threads = oracle_threads()
    lat = model.ladder(wl.L, wl.J_leg, wl.J_rung, W=wl.W)
    lay = model.layout(lat)
    sch = model.schedule(lat, lay)
    M = model.trotter_steps(wl.beta, wl.tau)
    gates = [model.gate(J, wl.tau / 2.0) for J in sch.couplings]
    swap = model.swap_gate()
    psi = mps.init_state(lay, mps.initial_outcomes(lay, wl.seed, 0), 0)
    st = mps.Stats()
    t0 = time.perf_counter()
    n = 0
    for u in model.evolve_updates(sch, M):
        if u.op == model.OP_SWAP:
            mps.apply_update(psi, u.k, swap, False, u.right, wl.chi_max,
                             wl.cutoff, st)
        else:
            mps.apply_update(psi, u.k, gates[u.op], True, u.right,
                             wl.chi_max, wl.cutoff, st)
        n += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    total = M * len(sch.step)
    return {"value": n / dt, "unit": UNIT, "cores": int(threads),
            "kind": "oracle", "n_updates": n,
            "sample": (f"first {n} of the {total} Trotter updates of sample 0 "
                       f"(chain 0, seed {wl.seed}); chi reached "
                       f"{st.max_chi} of {wl.chi_max}; the rest of the "
                       "sample runs at larger chi, so this rate is an upper "
                       "bound for the oracle")}


def svd_roofline(wl, s0, s1, use_traffic):
    """Roofline object of the round kernel over the timed region."""
    launches = s1.round_launches - s0.round_launches
    svd_s = s1.svd_seconds - s0.svd_seconds
    svd_f = s1.svd_flops - s0.svd_flops
    svd_b = s1.svd_bytes - s0.svd_bytes
    achieved = (svd_f / svd_s / 1e12) if svd_s > 0 else 0.0
    return {
        "bound": "mfma", "achieved": achieved,
        "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": achieved / FP64_PEAK_TFLOPS,
        "traffic": measured_traffic(wl) if use_traffic else None,
        "kernel": "k_jacobi_round",
        "launches": launches,
        "avg_launch_us": 1e6 * svd_s / launches if launches else None,
        "flops_per_launch": svd_f / launches if launches else None,
        "algo_bytes_per_launch": svd_b / launches if launches else None,
        "algo_hbm_GBps": svd_b / svd_s / 1e9 if svd_s > 0 else None,
        "hbm_peak_GBps": 8000.0,
    }


def oracle_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([p.get("num_threads", 1) for p in threadpool_info()]
                       or [1]))
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline_bond(wl, center, right, seconds):
    """The FP64 oracle's two-site update on chain 0's bond, repeated with
    the centre sweeping back and forth until the time budget is spent."""
    import numpy as np
    from oracle import model, mps
    tensors = [np.ascontiguousarray(T.transpose(1, 0, 2))   # [a, s, b]
               for T in (center[0], right[0])]
    psi = mps.MPS(tensors, 0)
    g = model.gate(wl.J, wl.x)
    t0 = time.perf_counter()
    n = 0
    while True:
        mps.apply_update(psi, 0, g, True, n % 2 == 0, wl.chi_max, wl.cutoff)
        n += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": UNIT, "cores": oracle_threads(),
            "kind": "oracle",
            "sample": (f"{n} gate applications on chain 0's bond (chi "
                       f"{wl.chi} x {wl.chi} x {wl.chi}, the same input) in "
                       f"{dt:.1f} s")}


def main_bond(args):
    """Single gate applications at chi = 256 (the m1 workload)."""
    import torch
    from paper_1910_09142_amd import hmps, workloads
    wl = workloads.M1
    B = args.chains or 1
    chi = wl.chi
    center, right = workloads.bond_tensors(wl.seed, B, chi, chi, chi,
                                           wl.decay)
    precision = (hmps.PREC_MIXED_FP32 if args.precision == "mixed"
                 else hmps.PREC_FP64)
    ctx = hmps.Context(B, 2, chi, 1, precision=precision)
    ctx.hmps_load_bond(center, right)
    for i in range(args.warmup):
        ctx.hmps_apply_gate(wl.J, wl.x, wl.chi_max, wl.cutoff)
    print(f"warmup done ({args.warmup} gate applications)", file=sys.stderr,
          flush=True)
    s0 = ctx.hmps_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ctx.hmps_apply_gate(wl.J, wl.x, wl.chi_max, wl.cutoff)
        if (i + 1) % 10 == 0:
            print(f"gate application {i + 1}/{args.steps} "
                  f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
                  flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s1 = ctx.hmps_stats()
    chi_now = ctx.hmps_bond_dims()[:, 1]
    ctx.hmps_destroy()
    gates = s1.gate_updates - s0.gate_updates
    out = {
        "metric": METRIC, "value": gates / elapsed, "unit": UNIT,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (Philox-seeded Haar bond tensors)",
        "config": {"workload": wl.name, "n_chains": B, "chi_l": chi,
                   "chi_m": chi, "chi_r": chi, "J": wl.J, "x": wl.x,
                   "chi_max": wl.chi_max, "cutoff": wl.cutoff,
                   "schmidt_decay": wl.decay, "precision": args.precision},
        "bond_dim_after": int(chi_now.min()),
        "algo_tflops": (s1.algo_flops - s0.algo_flops) / elapsed / 1e12,
        "jacobi_sweeps": s1.jacobi_sweeps - s0.jacobi_sweeps,
        "roofline": svd_roofline(wl, s0, s1, args.precision == "fp64"),
    }
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline_bond(wl, center, right,
                                                args.cpu_seconds)
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the chains are independent "
              "Markov chains that shard over GPUs without communication, and "
              "this benchmark does not run on more than one GPU",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "m1":
        main_bond(args)
        return
    import torch
    from paper_1910_09142_amd import hmps, workloads

    wl = getattr(workloads, args.workload.upper())
    B = args.chains or wl.n_chains
    n, bonds, order, mask = workloads.ladder_arrays(wl.L, wl.J_leg,
                                                    wl.J_rung, wl.W)
    lat = hmps.Lattice(n, bonds, order, mask)
    t_start = time.perf_counter()
    step_marks = []  # (Trotter steps done, time) of the first timed sample

    def progress(done, total):
        # one line per Trotter step: evolutions at chi = 256 take minutes
        now = time.perf_counter()
        step_marks.append((done, now))
        print(f"trotter step {done}/{total} ({now - t_start:.1f} s)",
              file=sys.stderr, flush=True)

    precision = (hmps.PREC_MIXED_FP32 if args.precision == "mixed"
                 else hmps.PREC_FP64)
    ctx = hmps.Context(B, workloads.mps_length(wl.L, wl.W), wl.chi_max,
                       len(bonds), precision=precision, progress=progress)
    ctx.hmps_init_cluster_env(lat, B, wl.seed)

    def one_sample(idx):
        ctx.hmps_evolve(wl.beta, wl.tau, wl.chi_max, wl.cutoff)
        m = ctx.hmps_measure()
        ctx.hmps_collapse_resample(idx % 2)
        return m

    sample = 0
    for _ in range(args.warmup):
        one_sample(sample)
        sample += 1
        print(f"warmup sample done", file=sys.stderr, flush=True)
    s0 = ctx.hmps_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    energies = []
    timed_marks = None
    for _ in range(args.steps):
        step_marks.clear()
        m = one_sample(sample)
        if timed_marks is None:
            timed_marks = list(step_marks)
        energies += m["energy"].tolist()
        sample += 1
        print(f"timed sample done ({time.perf_counter() - t0:.1f} s)",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s1 = ctx.hmps_stats()
    trotter_updates = ((s1.updates - s0.updates)
                       - (s1.move_updates - s0.move_updates))
    gates = s1.gate_updates - s0.gate_updates
    value = trotter_updates / elapsed
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (Philox-seeded product states, ladder Hamiltonian)",
        "config": {"workload": wl.name, "n_chains": B, "L": wl.L, "W": wl.W,
                   "J_leg": wl.J_leg, "J_rung": wl.J_rung, "beta": wl.beta,
                   "tau": wl.tau, "chi_max": wl.chi_max, "cutoff": wl.cutoff,
                   "samples_per_step": 1, "precision": args.precision},
        "samples_per_s": B * args.steps / elapsed,
        "hamiltonian_gates_per_s": gates / elapsed,
        "algo_tflops": (s1.algo_flops - s0.algo_flops) / elapsed / 1e12,
        "max_chi": s1.max_chi,
        "jacobi_sweeps": s1.jacobi_sweeps - s0.jacobi_sweeps,
        "energy_mean": sum(energies) / len(energies),
        "roofline": svd_roofline(
            wl, s0, s1, args.precision == "fp64" and B == wl.n_chains),
    }
    ctx.hmps_destroy()
    if args.cpu_seconds > 0:
        cb = cpu_baseline(wl, args.cpu_seconds)
        # the oracle covers only the first updates of the sample (small chi):
        # the GPU's rate over the same leading Trotter steps, for comparison
        per_step = trotter_updates / max(1, args.steps) / max(
            1, model_steps(wl))
        g = (prefix_rate(timed_marks or [], t0, cb["n_updates"], per_step)
             if B == 1 else None)
        if g is not None:
            cb["sample"] += (f"; the GPU ran the first {g[0]} Trotter steps "
                             f"of the timed sample ({g[1]} updates) at "
                             f"{g[2]:.1f} updates/s")
        del cb["n_updates"]
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
