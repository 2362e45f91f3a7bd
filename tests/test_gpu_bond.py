"""One gate application on a loaded bond (hmps_load_bond, hmps_apply_gate,
hmps_read_site) against the oracle's two-site update on the same tensors.

The update is the one every Trotter gate runs (Ancilla Method subsection):
theta = T_0 T_1, theta' = G theta, log ||theta'||^2 into the log-weight,
theta' normalised, truncated SVD (Results section: chi_max and the cutoff).
Inputs: the synthetic bond of the chi = 256 gate workload (Haar factors,
Schmidt values exp(-j/24)) at several sizes, so that theta' takes the
in-LDS SVD (m n <= 2048) and the blocked rounds (several 16-vector blocks
and a ragged tail).

Compared (gauge-invariant, FP64): bond dimensions exactly; the two-site
state T_0 T_1 after each application to 1e-10 relative (Frobenius), the
log-weight of the first application to 1e-12 absolute (ln ||theta'||^2 is
summed from theta' itself in FP64, before the SVD; later applications
start from states that already differ at the 1e-13 level, so they are held
at 1e-10); the factor left of the centre left-orthonormal and the one
right of it right-orthonormal, both to 1e-12 (one factor is the
normalised Jacobi vectors, or on the two-QR path their images under the
stored reflectors; the other their projections, corrected to
orthonormality).  Every preconditioning level is run (none, one QR, two).
Mixed mode (FP32 theta and gate): the state to 5e-6 relative, log-weights
to 1e-6.
"""
import ctypes

import numpy as np
import pytest

from oracle import model, mps
from paper_1910_09142_amd import hmps, workloads

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def to_oracle(T):
    """[s, a, b] (C ABI) -> [a, s, b] (oracle)."""
    return np.ascontiguousarray(T.transpose(1, 0, 2))


def state(T0, T1):
    """Two-site state as a (3 chi_l) x (3 chi_r) matrix, rows (a, s)."""
    l, r = T0.shape[1], T1.shape[2]
    return np.einsum("sab,tbc->astc", T0, T1).reshape(3 * l, 3 * r)


def oracle_state(psi):
    A, B = psi.tensors
    return np.einsum("asb,btc->astc", A, B).reshape(A.shape[0] * 3, -1)


def run_case(chi_l, chi_m, chi_r, n_chains, chi_max, cutoff, n_apply,
             precision=hmps.PREC_FP64, J=1.0, x=0.025, seed=3,
             tol_state=1e-10, tol_logw=1e-12, wide=None, width_rule=None):
    """wide: None, or whether the rounds must have taken wide blocks;
    width_rule: the context's width rule (None: the default)."""
    print(f"case: bond {chi_l}x{chi_m}x{chi_r}, {n_chains} chains, "
          f"chi_max {chi_max}, precision {precision}", flush=True)
    center, right = workloads.bond_tensors(seed, n_chains, chi_l, chi_m,
                                           chi_r)
    cap = max(chi_l, chi_m, chi_r, chi_max)
    ctx = hmps.Context(n_chains, 2, cap, 1, precision=precision,
                       width_rule=width_rule)
    ctx.hmps_load_bond(center, right)
    psis = [mps.MPS([to_oracle(center[c]), to_oracle(right[c])], 0)
            for c in range(n_chains)]
    g = model.gate(J, x)
    for it in range(n_apply):
        go_right = it % 2 == 0
        logw = ctx.hmps_apply_gate(J, x, chi_max, cutoff, want_logw=True)
        chi = ctx.hmps_bond_dims()
        for c in range(n_chains):
            S = mps.apply_update(psis[c], 0, g, True, go_right, chi_max,
                                 cutoff)
            A, B = psis[c].tensors
            assert chi[c].tolist() == [chi_l, A.shape[2], chi_r], (it, c)
            T0 = ctx.hmps_read_site(c, 0)
            T1 = ctx.hmps_read_site(c, 1)
            want = oracle_state(psis[c])
            got = state(T0, T1)
            err = np.linalg.norm(got - want) / np.linalg.norm(want)
            assert err < tol_state, (it, c, err)
            tl = tol_logw if it == 0 else max(tol_logw, 1e-10)
            assert abs(logw[c] - psis[c].logw) < tl, (it, c)
            k = T0.shape[2]
            if go_right:   # T0 left-orthonormal: rows (a, s)
                U = T0.transpose(1, 0, 2).reshape(-1, k)
                iso = U.T @ U
            else:          # T1 right-orthonormal: columns (s, c)
                V = T1.transpose(1, 0, 2).reshape(k, -1)
                iso = V @ V.T
            assert np.abs(iso - np.eye(k)).max() < 1e-12, (it, c)
    if wide is not None:
        assert (ctx.hmps_stats().wide_launches > 0) == wide
    ctx.hmps_destroy()


def test_in_lds_path_three_applications():
    # theta' 24 x 27 = 648 entries: the single-workgroup SVD
    run_case(8, 10, 9, 2, 16, 1e-10, 3)


def test_blocked_path_truncating():
    # theta' 120 x 120: eight 16-vector blocks with a ragged tail, chi_max
    # binds (40 -> 32)
    run_case(40, 40, 40, 3, 32, 1e-10, 3)


def test_blocked_path_wide():
    # more columns than rows: the SVD orthogonalises the 66 rows
    run_case(22, 50, 60, 2, 50, 1e-12, 2)


def test_chi256_gate_workload():
    wl = workloads.M1
    run_case(wl.chi, wl.chi, wl.chi, 2, wl.chi_max, wl.cutoff, 2, J=wl.J,
             x=wl.x)


def test_chi512_largest_bond():
    # the largest chi_max of the ladder workloads: theta' 1536 x 1536,
    # 96 blocks of 16 vectors, theta and write-back at full size
    run_case(512, 512, 512, 1, 512, 1e-10, 2, seed=11)


def test_wide_blocks_by_the_width_rule():
    # theta' 540 x 540 in 16 chains.  Under a rule {512 vectors: 16 chains}
    # the rounds take 32-vector blocks (18 of them, the last ragged), each
    # block pair one workgroup, and every chain matches the oracle to the
    # bars of the 16-wide rounds; a rule {512 vectors: 32 chains} keeps
    # them 16-wide, and so does the default (measured: 540 vectors take
    # wide blocks from 16 chains on) for a batch of 8
    run_case(180, 180, 180, 16, 180, 1e-10, 2, seed=13, wide=True,
             width_rule=[(512, 16)])
    run_case(180, 180, 180, 16, 180, 1e-10, 1, seed=13, wide=False,
             width_rule=[(512, 32)])
    run_case(180, 180, 180, 8, 180, 1e-10, 1, seed=13, wide=False)


def test_width_rule_is_checked():
    ctx = hmps.Context(2, 2, 8, 1)
    for bad in ([(500, 4)],                 # below 512 vectors
                [(768, 0)],                 # no chains
                [(768, 4), (600, 2)],       # nvec_min not ascending
                [(768, 4), (1024, 8)],      # chains_min increasing
                [(512 + i, 1) for i in range(17)]):   # too many entries
        with pytest.raises(hmps.HmpsError, match="status 1"):
            ctx.hmps_set_width_rule(bad)
    ctx.hmps_set_width_rule([(600, 32), (900, 8), (1500, 8)])
    ctx.hmps_set_width_rule([])             # the default again
    ctx.hmps_destroy()


def test_wide_blocks_follow_the_batch_size(monkeypatch):
    # HMPS_WIDE (read when a context is created): unset, the width rule (by
    # default 540 vectors take wide blocks from 16 chains on); 1 always (on
    # the FP64 paths from 512 vectors); 0 never
    run_case(180, 180, 180, 2, 180, 1e-10, 1, seed=13, wide=False)
    monkeypatch.setenv("HMPS_WIDE", "1")
    run_case(180, 180, 180, 2, 180, 1e-10, 2, seed=13, wide=True)
    run_case(256, 256, 256, 1, 200, 1e-10, 2, seed=5, wide=True)
    monkeypatch.setenv("HMPS_WIDE", "0")
    run_case(180, 180, 180, 16, 180, 1e-10, 1, seed=13, wide=False)


def test_wide_batch_is_bit_identical_to_single_chains(monkeypatch):
    # a chain's update depends on its own input and the block width only:
    # in a batch of 16 (wide under the rule {512: 16}) and alone with wide
    # blocks forced it gives the same bits
    chi, n = 180, 16
    center, right = workloads.bond_tensors(21, n, chi, chi, chi)
    ctx = hmps.Context(n, 2, chi, 1, width_rule=[(512, 16)])
    ctx.hmps_load_bond(center, right)
    ctx.hmps_apply_gate(1.0, 0.025, chi, 1e-10)
    assert ctx.hmps_stats().wide_launches > 0
    batch = [(ctx.hmps_read_site(c, 0), ctx.hmps_read_site(c, 1))
             for c in (0, 7, 15)]
    ctx.hmps_destroy()
    monkeypatch.setenv("HMPS_WIDE", "1")
    ctx = hmps.Context(1, 2, chi, 1)
    for i, c in enumerate((0, 7, 15)):
        ctx.hmps_load_bond(center[c:c + 1], right[c:c + 1])
        ctx.hmps_apply_gate(1.0, 0.025, chi, 1e-10)
        assert np.array_equal(ctx.hmps_read_site(0, 0), batch[i][0])
        assert np.array_equal(ctx.hmps_read_site(0, 1), batch[i][1])
    assert ctx.hmps_stats().wide_launches > 0
    ctx.hmps_destroy()


def test_short_rounds_in_a_large_batch_are_bit_identical_to_single_chains():
    # theta' 384 x 384 (two-QR path, R2^T of 384 rows) in 64 chains: 768
    # workgroups per round, so the 16-wide FP64 rounds take the register
    # budget of three workgroups per CU; alone, a chain's 12 workgroups take
    # the two-per-CU budget.  Both run the same arithmetic: same bits
    chi, n = 128, 64
    center, right = workloads.bond_tensors(23, n, chi, chi, chi)
    ctx = hmps.Context(n, 2, chi, 1)
    ctx.hmps_load_bond(center, right)
    ctx.hmps_apply_gate(1.0, 0.025, chi, 1e-10)
    assert ctx.hmps_stats().wide_launches == 0
    picks = (0, 31, 63)
    batch = [(ctx.hmps_read_site(c, 0), ctx.hmps_read_site(c, 1))
             for c in picks]
    ctx.hmps_destroy()
    ctx = hmps.Context(1, 2, chi, 1)
    for i, c in enumerate(picks):
        ctx.hmps_load_bond(center[c:c + 1], right[c:c + 1])
        ctx.hmps_apply_gate(1.0, 0.025, chi, 1e-10)
        assert np.array_equal(ctx.hmps_read_site(0, 0), batch[i][0]), c
        assert np.array_equal(ctx.hmps_read_site(0, 1), batch[i][1]), c
    ctx.hmps_destroy()


def test_wide_rounds_on_two_streams_are_bit_identical_to_one(monkeypatch):
    # 32 chains of theta' 540 x 540 take wide blocks (default rule) and,
    # at 9 block pairs each (288 workgroups a round), issue every round as
    # two dispatches of 16 chains on two streams; with HMPS_SPLIT=0 one
    # dispatch on one stream: same bits for every chain
    chi, n = 180, 32
    center, right = workloads.bond_tensors(29, n, chi, chi, chi)
    out = {}
    for split in ("1", "0"):
        monkeypatch.setenv("HMPS_SPLIT", split)
        ctx = hmps.Context(n, 2, chi, 1)
        ctx.hmps_load_bond(center, right)
        for _ in range(2):
            ctx.hmps_apply_gate(1.0, 0.025, chi, 1e-10)
        st = ctx.hmps_stats()
        assert st.wide_launches > 0
        assert (st.split_launches == st.wide_launches) == (split == "1")
        assert (st.split_launches == 0) == (split == "0")
        out[split] = [(ctx.hmps_read_site(c, 0), ctx.hmps_read_site(c, 1))
                      for c in range(n)]
        ctx.hmps_destroy()
    for c in range(n):
        assert np.array_equal(out["1"][c][0], out["0"][c][0]), c
        assert np.array_equal(out["1"][c][1], out["0"][c][1]), c


def test_mixed_precision_bond():
    run_case(64, 64, 64, 2, 64, 1e-10, 2, precision=hmps.PREC_MIXED_FP32,
             tol_state=5e-6, tol_logw=1e-6)


@pytest.mark.parametrize("level", ["0", "1", "2"])
def test_preconditioner_levels(level, monkeypatch):
    # HMPS_QR, read when a context is created, selects how the blocked
    # Jacobi SVD is preconditioned: none (rounds on theta'), one QR (rounds
    # on R^T), or two (the default from 160 vectors on: rounds on R2^T with
    # R^T = Q2 R2, the left factor from the stored reflectors).  Each level, in FP64 and in
    # mixed precision (FP32 rounds, FP64 Ritz step), gives the oracle's
    # update.
    monkeypatch.setenv("HMPS_QR", level)
    run_case(40, 40, 40, 3, 32, 1e-10, 3)
    run_case(22, 50, 60, 2, 50, 1e-12, 2)
    run_case(96, 96, 96, 1, 96, 1e-10, 2, seed=7)
    # wide and ragged with two QRs (180 vectors of length 240)
    run_case(60, 70, 80, 2, 70, 1e-10, 2, seed=9)
    run_case(64, 64, 64, 2, 64, 1e-10, 2, precision=hmps.PREC_MIXED_FP32,
             tol_state=5e-6, tol_logw=1e-6)


def test_identity_gate_keeps_the_state():
    # exp(0) = identity: theta' = theta, unit norm, nothing truncated
    chi = 12
    center, right = workloads.bond_tensors(5, 1, chi, chi, chi)
    ctx = hmps.Context(1, 2, chi, 1)
    ctx.hmps_load_bond(center, right)
    logw = ctx.hmps_apply_gate(1.0, 0.0, chi, 0.0, want_logw=True)
    got = state(ctx.hmps_read_site(0, 0), ctx.hmps_read_site(0, 1))
    want = state(center[0], right[0])
    ctx.hmps_destroy()
    assert np.linalg.norm(got - want) < 1e-12 * np.linalg.norm(want)
    assert abs(logw[0]) < 1e-13


def test_batch_is_bit_identical_to_single_chains():
    chi, n = 40, 3
    center, right = workloads.bond_tensors(9, n, chi, chi, chi)
    ctx = hmps.Context(n, 2, chi, 1)
    ctx.hmps_load_bond(center, right)
    for _ in range(2):
        ctx.hmps_apply_gate(1.0, 0.025, 32, 1e-10)
    batch = [(ctx.hmps_read_site(c, 0), ctx.hmps_read_site(c, 1))
             for c in range(n)]
    for c in range(n):
        ctx.hmps_load_bond(center[c:c + 1], right[c:c + 1])
        for _ in range(2):
            ctx.hmps_apply_gate(1.0, 0.025, 32, 1e-10)
        assert np.array_equal(ctx.hmps_read_site(0, 0), batch[c][0])
        assert np.array_equal(ctx.hmps_read_site(0, 1), batch[c][1])
    ctx.hmps_destroy()


def test_bond_entry_points_reject_bad_calls():
    ctx = hmps.Context(2, 2, 8, 1)
    with pytest.raises(hmps.HmpsError, match="status 4"):
        ctx.hmps_apply_gate(1.0, 0.1, 8, 0.0)        # nothing loaded
    center, right = workloads.bond_tensors(0, 1, 4, 12, 4)
    with pytest.raises(hmps.HmpsError, match="status 1"):
        ctx.hmps_load_bond(center, right)            # chi_m 12 > chi_cap 8
    center, right = workloads.bond_tensors(0, 1, 4, 8, 4)
    bad = center.copy()
    bad[0, 1, 2, 3] = np.nan
    with pytest.raises(hmps.HmpsError, match="status 1"):
        ctx.hmps_load_bond(bad, right)
    ctx.hmps_load_bond(center, right)
    with pytest.raises(hmps.HmpsError, match="status 1"):
        ctx.hmps_apply_gate(1.0, 0.1, 9, 0.0)        # chi_max > chi_cap
    with pytest.raises(hmps.HmpsError, match="status 1"):
        ctx.hmps_apply_gate(1.0, 0.1, 8, -1.0)       # negative cutoff
    out = np.zeros(3 * 4 * 8)
    ptr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert ctx.lib.hmps_read_site(ctx.h, 1, 0, ptr) == 1   # one chain only
    assert ctx.lib.hmps_read_site(ctx.h, 0, 2, ptr) == 1   # two sites only
    assert ctx.lib.hmps_read_site(ctx.h, 0, 0, None) == 1
    ctx.hmps_destroy()
