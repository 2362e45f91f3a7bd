#!/usr/bin/env python3
"""Benchmark of the hybrid METTS-ancilla hot path on one MI355X.

Default line: two-site gate applications per second at chi = 256, FP64,
64 independent chains batched.  Every chain holds one MPS bond with chi_l =
chi_m = chi_r = 256 (synthetic Haar factors, Schmidt values exp(-j/24));
one step applies exp(-(tau/2) J S.S) (tau = 0.05, J = 1) to every chain:
theta = T_k T_{k+1}, the gate, the log-weight update, and the truncated
SVD of the 768 x 768 theta' back to chi_max = 256 at cutoff 1e-10, the
bond swept back and forth (Ancilla Method subsection: a two-site gate
followed by a truncated SVD; Results section: the cutoff).  Inputs are
resident on the device before the timed region.

Extra fields of the same line: the same workload on one chain, in mixed
precision (FP32 theta and gate) with its speedup over FP64, a bounded
samples-per-second run (one full Markov-chain sample of 64 chains of the
2x8 ladder at beta = 1), the roofline of the dominant kernel and the FP64
oracle on the host's cores.

`--workload c1..c5` runs whole samples of a ladder workload instead (one
step = one sample of every chain: evolution to beta/2, measurement,
collapse), `--workload m1` the gate workload alone.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("two-site gate apps/sec at χ=256 (FP64 vs mixed, batched); "
          "METTS samples/sec")
UNIT = "two-site gate applications/s"
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBPS = 8000.0
DEFAULT_CHAINS = 64

# Conservative rates used only to check that a command's planned work fits
# the time the bench is given (half of what MI355X measured).
PLAN_GATES_PER_S_BATCHED = 150.0    # chi = 256, 64 chains
PLAN_GATES_PER_S_SINGLE = 12.0      # chi = 256, one chain
PLAN_SAMPLE_SECONDS = 60.0          # one 2x8 beta = 1 sample of 64 chains
PLAN_U1_SAMPLE_SECONDS = 30.0       # the same sample with U(1) updates
PLAN_STARTUP_SECONDS = 150.0        # first torch import on a fresh box,
                                    # inputs, library load


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="gate",
                    choices=["gate", "m1", "c1", "c2", "c3", "c4", "c5",
                             "wlimit"],
                    help="gate (default): the chi = 256 gate workload with "
                    "its extra fields; m1: that workload alone; c1..c5: "
                    "whole samples of a ladder workload; wlimit: the hybrid "
                    "against its METTS (W = 0) and ancilla (W = L) limits "
                    "(--steps samples per chain)")
    ap.add_argument("--chains", type=int, default=None,
                    help="chains (default: 64 for the gate workload, the "
                    "workload's own count for ladders)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="mixed: FP32 theta contraction and gate on the "
                    "matrix cores, FP64 SVD, truncation and observables")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget of the oracle baseline (0 disables it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="gate workload: headline measurement only")
    ap.add_argument("--beta", type=float, default=None,
                    help="ladder workloads: override beta")
    ap.add_argument("--symmetry", default="none", choices=["none", "u1"],
                    help="ladder workloads: u1 splits every update into its "
                    "charge blocks (every collapse in S^z)")
    ap.add_argument("--collapse", default="alternate",
                    choices=["alternate", "z"],
                    help="ladder workloads: collapse basis S^z / S^x by "
                    "sample parity, or S^z always (forced by --symmetry u1)")
    ap.add_argument("--window", default=None, metavar="START:COUNT",
                    help="ladder workloads: time Trotter steps START .. "
                    "START+COUNT-1 of the first evolution only (the steps "
                    "before run untimed); reports the bond-dimension "
                    "histogram at the end of the window")
    args = ap.parse_args(argv)
    if args.steps < 1 or args.warmup < 0:
        ap.error("--steps >= 1 and --warmup >= 0")
    if args.symmetry == "u1":
        args.collapse = "z"
    return args


def planned_seconds(args) -> float:
    """Upper estimate of the wall time of a command, from conservative
    rates: the bench must finish well inside the time it is given."""
    if args.workload not in ("gate", "m1"):
        return float("inf")    # whole ladder samples: minutes per step
    n = args.steps + args.warmup
    B = args.chains or DEFAULT_CHAINS
    rate = PLAN_GATES_PER_S_SINGLE if B == 1 else PLAN_GATES_PER_S_BATCHED
    t = PLAN_STARTUP_SECONDS + n * B / rate
    if args.workload == "gate" and not args.no_extras:
        t += n * B / PLAN_GATES_PER_S_BATCHED        # mixed, batched
        t += n / PLAN_GATES_PER_S_SINGLE              # one chain
        t += PLAN_SAMPLE_SECONDS + PLAN_U1_SAMPLE_SECONDS
    return t + args.cpu_seconds


# ---------------------------------------------------------------------------
# roofline
# ---------------------------------------------------------------------------
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


def measured_traffic(kernel, tag):
    """HBM bytes per launch of the round kernel `kernel` from the committed
    rocprofv3 counter summary of this workload (FETCH_SIZE and WRITE_SIZE
    scaled by the copy-kernel calibration), or None when there is none or
    it was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic_{tag}.md")
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


def svd_roofline(tag, s0, s1, use_traffic):
    """Roofline object of the round kernel over the timed region: achieved
    = Golub-Reinsch SVD flops of the updates (the algorithmic count) over
    the HIP-event span of the rounds on the library's stream."""
    launches = s1.round_launches - s0.round_launches
    wide = s1.wide_launches - s0.wide_launches
    # the rounds of these updates: all on 32-vector blocks, all on 16-wide
    # ones, or both (a batch with chains on either side of the width rule)
    kernel = ("k_jacobi_round_wide" if wide == launches else
              "k_jacobi_round" if wide == 0 else
              "k_jacobi_round+k_jacobi_round_wide")
    svd_s = s1.svd_seconds - s0.svd_seconds
    svd_f = s1.svd_flops - s0.svd_flops
    svd_b = s1.svd_bytes - s0.svd_bytes
    achieved = (svd_f / svd_s / 1e12) if svd_s > 0 else 0.0
    # a launch is one round over all chains; a split round is two
    # concurrent dispatches (the two halves of the chains, two streams),
    # and its time is the span of both
    split = s1.split_launches - s0.split_launches
    return {
        "bound": "mfma", "achieved": achieved,
        "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": achieved / FP64_PEAK_TFLOPS,
        "traffic": measured_traffic(kernel, tag) if use_traffic else None,
        "kernel": kernel,
        "launches": launches,
        "dispatches_per_launch": (2 if split == launches else
                                  1 if split == 0 else
                                  1 + split / launches) if launches else None,
        "avg_launch_us": 1e6 * svd_s / launches if launches else None,
        "flops_per_launch": svd_f / launches if launches else None,
        "algo_bytes_per_launch": svd_b / launches if launches else None,
        "algo_hbm_GBps": svd_b / svd_s / 1e9 if svd_s > 0 else None,
        "hbm_peak_GBps": HBM_PEAK_GBPS,
    }


# ---------------------------------------------------------------------------
# host description and the oracle baselines
# ---------------------------------------------------------------------------
def host_info():
    import numpy  # noqa: F401  (loads the BLAS threadpoolctl reports)
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas, threads = "unknown", os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        info = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        if info:
            blas = (f"{info[0].get('internal_api')} "
                    f"{info[0].get('version')}").strip()
            threads = int(info[0].get("num_threads", threads))
    except Exception:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(),
            "blas": blas, "blas_threads": threads}


def oracle_bond_rate(wl, center, right, seconds, threads=None):
    """The FP64 oracle's two-site update on chain 0's bond, repeated with
    the centre sweeping back and forth until the time budget is spent;
    returns (applications per second, applications, seconds)."""
    import numpy as np
    from oracle import model, mps
    tensors = [np.ascontiguousarray(T.transpose(1, 0, 2))   # [a, s, b]
               for T in (center[0], right[0])]
    psi = mps.MPS(tensors, 0)
    g = model.gate(wl.J, wl.x)

    def loop():
        t0 = time.perf_counter()
        n = 0
        while True:
            mps.apply_update(psi, 0, g, True, n % 2 == 0, wl.chi_max,
                             wl.cutoff)
            n += 1
            if time.perf_counter() - t0 > seconds:
                break
        return n, time.perf_counter() - t0

    if threads is None:
        n, dt = loop()
    else:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=threads):
            n, dt = loop()
    return n / dt, n, dt


def cpu_baseline_bond(wl, center, right, seconds):
    """The oracle on the gate workload: all BLAS threads for 2/3 of the
    budget, then one thread (the paper's one-core protocol) for the rest."""
    info = host_info()
    v_all, n_all, dt_all = oracle_bond_rate(wl, center, right,
                                            seconds * 2.0 / 3.0)
    v_one, n_one, dt_one = oracle_bond_rate(wl, center, right,
                                            seconds / 3.0, threads=1)
    return {"value": v_all, "unit": UNIT, "cores": info["blas_threads"],
            "kind": "oracle",
            "sample": (f"{n_all} gate applications on chain 0's bond (chi "
                       f"{wl.chi} x {wl.chi} x {wl.chi}, the GPU's input) in "
                       f"{dt_all:.1f} s on {info['blas_threads']} BLAS "
                       f"threads; then {n_one} in {dt_one:.1f} s on one "
                       "thread"),
            "single_core_value": v_one,
            **info}


# ---------------------------------------------------------------------------
# gate workload
# ---------------------------------------------------------------------------
def gate_run(wl, center, right, precision, steps, warmup, label):
    """Applies the gate steps + warmup times to every chain; returns the
    rate over the timed steps and the stats around them."""
    import torch
    from paper_1910_09142_amd import hmps
    B = center.shape[0]
    ctx = hmps.Context(B, 2, wl.chi, 1, precision=precision)
    ctx.hmps_load_bond(center, right)
    for _ in range(warmup):
        ctx.hmps_apply_gate(wl.J, wl.x, wl.chi_max, wl.cutoff)
    s0 = ctx.hmps_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ctx.hmps_apply_gate(wl.J, wl.x, wl.chi_max, wl.cutoff)
        if (i + 1) % 10 == 0 or i + 1 == steps:
            print(f"{label}: gate step {i + 1}/{steps} "
                  f"({time.perf_counter() - t0:.2f} s)", file=sys.stderr,
                  flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s1 = ctx.hmps_stats()
    chi_now = ctx.hmps_bond_dims()[:, 1]
    logw = ctx.hmps_apply_gate(wl.J, wl.x, wl.chi_max, wl.cutoff,
                               want_logw=True)
    ctx.hmps_destroy()
    gates = s1.gate_updates - s0.gate_updates
    return {"rate": gates / elapsed, "elapsed": elapsed, "s0": s0, "s1": s1,
            "chi_after": int(chi_now.min()), "logw": logw,
            "sweeps_per_gate": (s1.jacobi_sweeps - s0.jacobi_sweeps)
            / max(1, steps),
            "sweeps32_per_gate": (s1.jacobi_sweeps_fp32 - s0.jacobi_sweeps_fp32)
            / max(1, steps),
            "algo_tflops": (s1.algo_flops - s0.algo_flops) / elapsed / 1e12}


def sample_run(wl, B, precision, symmetry=0):
    """One full Markov-chain sample of B chains of a ladder workload:
    evolution to beta/2, measurement, collapse in S^z (timed from resident
    S^z product states); symmetry 1: U(1) block-sparse updates."""
    import torch
    from paper_1910_09142_amd import hmps, workloads
    n, bonds, order, mask = workloads.ladder_arrays(wl.L, wl.J_leg,
                                                    wl.J_rung, wl.W)
    lat = hmps.Lattice(n, bonds, order, mask)
    ctx = hmps.Context(B, workloads.mps_length(wl.L, wl.W), wl.chi_max,
                       len(bonds), precision=precision, symmetry=symmetry)
    ctx.hmps_init_cluster_env(lat, B, wl.seed)
    s0 = ctx.hmps_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.hmps_evolve(wl.beta, wl.tau, wl.chi_max, wl.cutoff)
    m = ctx.hmps_measure()
    ctx.hmps_collapse_resample(0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s1 = ctx.hmps_stats()
    ctx.hmps_destroy()
    ups = (s1.updates - s0.updates) - (s1.move_updates - s0.move_updates)
    return {"workload": wl.name, "n_chains": B, "samples": B,
            "seconds": elapsed, "value": B / elapsed,
            "unit": "METTS samples/s",
            "trotter_updates_per_s": ups / elapsed,
            "hamiltonian_gates_per_s": (s1.gate_updates - s0.gate_updates)
            / elapsed,
            "max_chi": s1.max_chi,
            "energy_mean": float(m["energy"].mean())}


def main_wlimit(args):
    """The hybrid against its two limits on one code path (Results
    section: the W = 16 hybrid against METTS and the ancilla method;
    Entanglement and Cost of Hybrid States: the variance of each bond
    energy along a leg).  A 2 x 8 S=1 ladder at beta = 2 (tau 0.05,
    chi_max 128, cutoff 1e-12) with cluster widths W = 0 (METTS), 2, 4
    (hybrid) and 8 (the ancilla method: one purified state, no sampling):
    per W the energy per site with its standard error over independent
    chains, the sample variance of every leg bond energy (device moments),
    the cost per sample and the largest bond dimension.  Every chain starts
    from a uniform random product state; its first --warmup samples are
    discarded (burn-in towards the stationary distribution P_i / sum P_j)
    and the next --steps are measured.  --symmetry u1 runs the hybrid and
    ancilla points with U(1) block-sparse updates and every collapse in
    S^z (Exploiting Conserved Quantum Numbers subsection); METTS keeps the
    dense path and the alternating bases, since S^z collapses of every site
    would keep it in one sector of the total S^z."""
    import numpy as np
    import torch
    from paper_1910_09142_amd import hmps, workloads
    L, beta, tau, chi, cut = 8, (args.beta or 2.0), 0.05, 128, 1e-12
    B, S, burn = (args.chains or 64), args.steps, args.warmup
    rows = []
    t_all = time.perf_counter()
    for W in (0, 2, 4, L):
        # the ancilla limit samples nothing: one purified state
        nc, ns, nb = (1, 1, 0) if W == L else (B, S, burn)
        n, bonds, order, mask = workloads.ladder_arrays(L, 1.0, 1.0, W)
        lat = hmps.Lattice(n, bonds, order, mask)
        u1 = args.symmetry == "u1" and W > 0
        ctx = hmps.Context(nc, workloads.mps_length(L, W), chi, len(bonds),
                           symmetry=hmps.SYM_U1 if u1 else hmps.SYM_NONE)
        ctx.hmps_init_cluster_env(lat, nc, 0)
        e = np.zeros((nc, ns))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(nb + ns):
            ctx.hmps_evolve(beta, tau, chi, cut)
            if k >= nb:
                m = ctx.hmps_measure(hmps.MEASURE_ENERGY |
                                     hmps.MEASURE_ACCUMULATE)
                e[:, k - nb] = m["energy"] / n
            ctx.hmps_collapse_resample(0 if u1 else k % 2)
            print(f"wlimit W={W}: sample {k + 1}/{nb + ns} "
                  f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.hmps_stats()
        leg = slice(L, 2 * L - 1)   # bonds (c, 0)-(c + 1, 0)
        var = None
        if nc * ns >= 2:
            var = ctx.hmps_bond_moments()["var"][leg].tolist()
        ctx.hmps_destroy()
        means = e.mean(axis=1)       # per chain: chains are independent
        se = float(means.std(ddof=1) / np.sqrt(nc)) if nc > 1 else 0.0
        rows.append({"W": W, "method": ("METTS" if W == 0 else "ancilla"
                                        if W == L else "hybrid"),
                     "symmetry": "u1" if u1 else "none",
                     "chains": nc, "samples_per_chain": ns,
                     "burn_in_per_chain": nb,
                     "energy_per_site": float(means.mean()),
                     "standard_error": se,
                     "leg_bond_variance": var,
                     "seconds": dt, "samples_per_s": nc * (nb + ns) / dt,
                     "max_chi": st.max_chi})
    ref = rows[-1]["energy_per_site"]
    for r in rows:
        r["minus_ancilla"] = r["energy_per_site"] - ref
    hyb = rows[2]
    out = {
        "metric": "METTS samples/sec, hybrid vs METTS vs ancilla limits",
        "value": hyb["samples_per_s"], "unit": "METTS samples/s",
        "n_gpus": 1, "steps": S, "warmup": burn,
        "ms_per_step": 1e3 * hyb["seconds"] / (S + burn),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (Philox-seeded product states, "
        "ladder Hamiltonian)",
        "config": {"workload": f"ladder2x{L}_beta{beta:g}_chi{chi}_Wlimits",
                   "n_chains": B, "L": L, "beta": beta, "tau": tau,
                   "chi_max": chi, "cutoff": cut, "W": [0, 2, 4, L],
                   "symmetry": args.symmetry},
        "wlimit": rows, "seconds_total": time.perf_counter() - t_all}
    print(json.dumps(out), flush=True)


def gate_tag(wl, B):
    return wl.name if B == 1 else f"{wl.name}_batch{B}"


def main_gate(args, extras):
    """Gate applications at chi = 256 (the headline line)."""
    import numpy as np
    from paper_1910_09142_amd import hmps, workloads
    wl = workloads.M1
    B = args.chains or DEFAULT_CHAINS
    center, right = workloads.bond_tensors(wl.seed, B, wl.chi, wl.chi,
                                           wl.chi, wl.decay)
    prec = (hmps.PREC_MIXED_FP32 if args.precision == "mixed"
            else hmps.PREC_FP64)
    copy_probe()
    print(f"inputs ready: {B} bonds at chi {wl.chi}", file=sys.stderr,
          flush=True)
    head = gate_run(wl, center, right, prec, args.steps, args.warmup,
                    f"{args.precision} x{B}")
    tag = gate_tag(wl, B)
    out = {
        "metric": METRIC, "value": head["rate"], "unit": UNIT,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * head["elapsed"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (Philox-seeded Haar bond tensors)",
        "config": {"workload": tag, "n_chains": B, "chi_l": wl.chi,
                   "chi_m": wl.chi, "chi_r": wl.chi, "J": wl.J, "x": wl.x,
                   "chi_max": wl.chi_max, "cutoff": wl.cutoff,
                   "schmidt_decay": wl.decay, "precision": args.precision},
        "bond_dim_after": head["chi_after"],
        "algo_tflops": head["algo_tflops"],
        "jacobi_sweeps_per_gate": head["sweeps_per_gate"],
        "roofline": svd_roofline(tag, head["s0"], head["s1"],
                                 args.precision == "fp64"),
    }
    if extras:
        one = gate_run(wl, center[:1], right[:1], prec, args.steps,
                       args.warmup, f"{args.precision} x1")
        out["single_chain"] = {
            "value": one["rate"], "unit": UNIT,
            "ms_per_gate": 1e3 / one["rate"],
            "jacobi_sweeps_per_gate": one["sweeps_per_gate"],
            "roofline": svd_roofline(gate_tag(wl, 1), one["s0"], one["s1"],
                                     False)}
        other = "mixed" if args.precision == "fp64" else "fp64"
        oprec = (hmps.PREC_MIXED_FP32 if other == "mixed"
                 else hmps.PREC_FP64)
        alt = gate_run(wl, center, right, oprec, args.steps, args.warmup,
                       f"{other} x{B}")
        fp64, mixed = (head, alt) if other == "mixed" else (alt, head)
        out["mixed"] = {
            "value": mixed["rate"], "unit": UNIT, "n_chains": B,
            "speedup_vs_fp64": mixed["rate"] / fp64["rate"],
            "jacobi_sweeps_per_gate": mixed["sweeps_per_gate"],
            "fp32_sweeps_per_gate": mixed["sweeps32_per_gate"],
            "max_abs_logw_diff_vs_fp64": float(
                np.abs(mixed["logw"] - fp64["logw"]).max())}
        c2 = dataclasses.replace(workloads.C2, beta=1.0,
                                 name="ladder2x8_W2_beta1_chi128")
        out["samples_per_s"] = sample_run(c2, DEFAULT_CHAINS, prec)
        print("sample run done", file=sys.stderr, flush=True)
        if args.precision == "fp64":
            # the same sample with U(1) block-sparse updates (Exploiting
            # Conserved Quantum Numbers subsection)
            u1 = sample_run(c2, DEFAULT_CHAINS, prec, hmps.SYM_U1)
            u1["speedup_vs_dense"] = (u1["value"] /
                                      out["samples_per_s"]["value"])
            u1["energy_mean_diff_vs_dense"] = abs(
                u1["energy_mean"] - out["samples_per_s"]["energy_mean"])
            out["samples_per_s_u1"] = u1
            print("U(1) sample run done", file=sys.stderr, flush=True)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline_bond(wl, center, right,
                                                args.cpu_seconds)
    print(json.dumps(out), flush=True)


def copy_probe():
    """One device-to-device copy of 256 MiB: the calibration kernel of the
    hardware byte counters in a profiled run of this command."""
    import torch
    a = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


# ---------------------------------------------------------------------------
# whole samples of a ladder workload
# ---------------------------------------------------------------------------
def main_window(args, wl, B, ctx):
    """Trotter steps START .. START+COUNT-1 of the first evolution of B
    chains, timed; the bond dimensions of every chain afterwards."""
    import numpy as np
    import torch
    from paper_1910_09142_amd import hmps
    start, count = (int(x) for x in args.window.split(":"))
    n, steps = hmps.hmps_schedule(ctx._lat)
    per = len(steps)
    M = int(round(wl.beta / (2.0 * wl.tau)))
    if start < 0 or count < 1 or start + count > M:
        raise SystemExit(f"--window outside the {M} Trotter steps")
    ctx.hmps_evolve_updates(wl.beta, wl.tau, wl.chi_max, wl.cutoff, 0,
                            start * per)
    s0 = ctx.hmps_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(count):
        ctx.hmps_evolve_updates(wl.beta, wl.tau, wl.chi_max, wl.cutoff,
                                (start + i) * per, per)
        print(f"window step {start + i + 1} ({time.perf_counter() - t0:.1f} s)",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s1 = ctx.hmps_stats()
    chi = ctx.hmps_bond_dims()
    # bonds inside the chain (the two open ends have dimension 1)
    inner = chi[:, 1:-1].ravel()
    edges = [1, 2, 4, 8, 16, 32, 64, 128, 192, 256, 384, 512, 1 << 30]
    hist = {f"{edges[i]}-{edges[i + 1] - 1}": int(((inner >= edges[i]) &
                                                   (inner < edges[i + 1])).sum())
            for i in range(len(edges) - 1)
            if ((inner >= edges[i]) & (inner < edges[i + 1])).any()}
    ups = s1.updates - s0.updates - (s1.move_updates - s0.move_updates)
    gates = s1.gate_updates - s0.gate_updates
    out = {
        "metric": METRIC, "value": gates / elapsed, "unit": UNIT,
        "n_gpus": 1, "steps": count, "warmup": start,
        "ms_per_step": 1e3 * elapsed / count, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (Philox-seeded product states, ladder Hamiltonian)",
        "config": {"workload": f"{wl.name}_chains{B}_steps{start}-"
                   f"{start + count - 1}", "n_chains": B, "L": wl.L,
                   "W": wl.W, "J_leg": wl.J_leg, "J_rung": wl.J_rung,
                   "beta": wl.beta, "tau": wl.tau, "chi_max": wl.chi_max,
                   "cutoff": wl.cutoff, "trotter_steps": [start, start + count],
                   "precision": args.precision, "symmetry": args.symmetry},
        "trotter_updates_per_s": ups / elapsed,
        "algo_tflops": (s1.algo_flops - s0.algo_flops) / elapsed / 1e12,
        "chi_histogram_after": hist,
        "chi_mean_after": float(inner.mean()),
        "max_chi": int(inner.max()),
        "jacobi_sweeps": s1.jacobi_sweeps - s0.jacobi_sweeps,
        "u1_blocks": s1.u1_blocks - s0.u1_blocks,
        "roofline": svd_roofline(wl.name, s0, s1, False),
    }
    print(json.dumps(out), flush=True)


def qn_histogram(charges):
    """{Q: count} of the samples whose <Q> is an integer to 1e-6, and the
    count of the others (S^x environments have no definite Q)."""
    hist, other = {}, 0
    for q in charges:
        r = round(q)
        if abs(q - r) <= 1e-6:
            hist[str(r)] = hist.get(str(r), 0) + 1
        else:
            other += 1
    out = dict(sorted(hist.items(), key=lambda kv: int(kv[0])))
    if other:
        out["not_integer"] = other
    return out


def main_ladder(args):
    import torch
    from paper_1910_09142_amd import hmps, workloads

    wl = getattr(workloads, args.workload.upper())
    if args.beta is not None:
        wl = dataclasses.replace(wl, beta=args.beta,
                                 name=f"{wl.name}_beta{args.beta:g}")
    B = args.chains or wl.n_chains
    n, bonds, order, mask = workloads.ladder_arrays(wl.L, wl.J_leg,
                                                    wl.J_rung, wl.W)
    lat = hmps.Lattice(n, bonds, order, mask)
    t_start = time.perf_counter()

    def progress(done, total):
        print(f"trotter step {done}/{total} "
              f"({time.perf_counter() - t_start:.1f} s)", file=sys.stderr,
              flush=True)

    precision = (hmps.PREC_MIXED_FP32 if args.precision == "mixed"
                 else hmps.PREC_FP64)
    symmetry = hmps.SYM_U1 if args.symmetry == "u1" else hmps.SYM_NONE
    ctx = hmps.Context(B, workloads.mps_length(wl.L, wl.W), wl.chi_max,
                       len(bonds), precision=precision, progress=progress,
                       symmetry=symmetry)
    ctx.hmps_init_cluster_env(lat, B, wl.seed)
    if args.window:
        main_window(args, wl, B, ctx)
        ctx.hmps_destroy()
        return

    def one_sample(idx):
        ctx.hmps_evolve(wl.beta, wl.tau, wl.chi_max, wl.cutoff)
        m = ctx.hmps_measure()
        ctx.hmps_collapse_resample(0 if args.collapse == "z" else idx % 2)
        return m

    sample = 0
    for _ in range(args.warmup):
        one_sample(sample)
        sample += 1
    s0 = ctx.hmps_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    energies, charges = [], []
    for _ in range(args.steps):
        m = one_sample(sample)
        energies += m["energy"].tolist()
        charges += m["qn"].tolist()
        sample += 1
        print(f"timed sample done ({time.perf_counter() - t0:.1f} s)",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s1 = ctx.hmps_stats()
    ctx.hmps_destroy()
    trotter_updates = ((s1.updates - s0.updates)
                       - (s1.move_updates - s0.move_updates))
    gates = s1.gate_updates - s0.gate_updates
    out = {
        "metric": METRIC, "value": gates / elapsed, "unit": UNIT,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (Philox-seeded product states, ladder Hamiltonian)",
        "config": {"workload": wl.name if B == wl.n_chains
                   else f"{wl.name}_chains{B}",
                   "n_chains": B, "L": wl.L, "W": wl.W,
                   "J_leg": wl.J_leg, "J_rung": wl.J_rung, "beta": wl.beta,
                   "tau": wl.tau, "chi_max": wl.chi_max, "cutoff": wl.cutoff,
                   "samples_per_step": 1, "precision": args.precision,
                   "symmetry": args.symmetry, "collapse": args.collapse},
        "samples_per_s": B * args.steps / elapsed,
        "trotter_updates_per_s": trotter_updates / elapsed,
        "algo_tflops": (s1.algo_flops - s0.algo_flops) / elapsed / 1e12,
        "max_chi": s1.max_chi,
        "jacobi_sweeps": s1.jacobi_sweeps - s0.jacobi_sweeps,
        "u1_blocks": s1.u1_blocks - s0.u1_blocks,
        "energy_mean": sum(energies) / len(energies),
        # the total S^z of the timed samples (an integer when the
        # environment was collapsed in S^z; Exploiting Conserved Quantum
        # Numbers subsection: it fluctuates from sample to sample)
        "qn_histogram": qn_histogram(charges),
        "roofline": svd_roofline(wl.name, s0, s1,
                                 args.precision == "fp64" and
                                 B == wl.n_chains and
                                 args.symmetry == "none"),
    }
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
    if args.workload in ("gate", "m1"):
        main_gate(args, extras=args.workload == "gate" and not args.no_extras)
    elif args.workload == "wlimit":
        main_wlimit(args)
    else:
        main_ladder(args)


if __name__ == "__main__":
    main()
