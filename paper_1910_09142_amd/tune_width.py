"""Measures the block-width rule of the Jacobi rounds on this GPU.

The blocked Jacobi SVD rotates pairs of 16-vector blocks, or of 32-vector
blocks for large FP64 updates in large batches (hmps_set_width_rule in
include/hmps.h).  A wide block pair is four times the work of a 16-wide one
on a single compute unit, in half as many workgroups, so which width is
faster depends on the size of theta' and on the number of chains.  This
script times gate applications on the synthetic bond of the gate workload
(Haar factors, Schmidt values exp(-j/24)) with chi_l = chi_m = chi_r = chi
(3 chi vectors) for a grid of chi and batch sizes, once with each width
(HMPS_WIDE=0 and 1 at create time), and writes

    {"device": ..., "measured": {chi: {chains: [rate_16, rate_wide]}},
     "rule": [[nvec_min, chains_min], ...]}

to width_rule_gfx950.json beside this file.  An entry (3 chi, b) means
wide blocks from b chains on; b is the smallest measured batch size from
which the wide rounds are faster at every larger measured size.  The
entries are made monotone (a larger theta' never needs more chains).  The
library's default rule is the table this script measured on MI355X (the
committed width_rule_gfx950.json); Context(width_rule=...) or
hmps_set_width_rule applies another.

    python -m paper_1910_09142_amd.tune_width [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "width_rule_gfx950.json")


def rate(hmps, workloads, chi, B, wide, steps):
    """Gate applications per second with the width forced."""
    import torch
    os.environ["HMPS_WIDE"] = "1" if wide else "0"
    try:
        center, right = workloads.bond_tensors(7, B, chi, chi, chi, 24.0)
        ctx = hmps.Context(B, 2, chi, 1)
        ctx.hmps_load_bond(center, right)
        ctx.hmps_apply_gate(1.0, 0.025, chi, 1e-10)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.hmps_apply_gate(1.0, 0.025, chi, 1e-10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.hmps_destroy()
    finally:
        del os.environ["HMPS_WIDE"]
    return B * steps / dt


def derive_rule(measured):
    rule = []
    for chi in sorted(measured):
        runs = measured[chi]
        sizes = sorted(runs)
        best = None
        for i, b in enumerate(sizes):
            if all(runs[c][1] > runs[c][0] for c in sizes[i:]):
                best = b
                break
        if best is None:
            continue
        if rule and best > rule[-1][1]:
            best = rule[-1][1]
        if 3 * chi >= 512:
            rule.append([3 * chi, best])
    return rule


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--quick", action="store_true",
                    help="two sizes and fewer batch sizes")
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    from paper_1910_09142_amd import hmps, workloads
    chis = [180, 256] if args.quick else [180, 256, 384, 512]
    batches = [2, 8, 16, 32, 64] if args.quick else [1, 2, 4, 8, 16, 32, 64]
    measured = {}
    for chi in chis:
        measured[chi] = {}
        steps = 3 if chi <= 256 else 2
        for B in batches:
            r16 = rate(hmps, workloads, chi, B, False, steps)
            rw = rate(hmps, workloads, chi, B, True, steps)
            measured[chi][B] = [r16, rw]
            print(f"chi {chi} ({3 * chi} vectors), {B} chains: 16-wide "
                  f"{r16:.1f}, wide {rw:.1f} gate applications/s",
                  flush=True)
    out = {"device": torch.cuda.get_device_name(0),
           "measured": {str(c): {str(b): v for b, v in m.items()}
                        for c, m in measured.items()},
           "rule": derive_rule(measured)}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["rule"]), flush=True)


if __name__ == "__main__":
    main()
