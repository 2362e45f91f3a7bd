"""Pins of the FP64 oracle against closed forms, library routines, brute
force and identities of the method (CPU only).

Each test names what fixes the expected value; none of them re-types the
oracle's own formula.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import exact, hybrid, model, mps, philox


# --------------------------------------------------------------------------
# gate
# --------------------------------------------------------------------------
@pytest.mark.parametrize("J,x", [(1.0, 0.025), (0.5, 0.05), (1.3, 0.7),
                                 (-0.4, 0.3)])
def test_gate_matches_expm(J, x):
    h = exact.bond_operator(0, 1, 2)
    ref = scipy.linalg.expm(-x * J * h)
    assert np.abs(model.gate(J, x) - ref).max() < 1e-14


def test_gate_conserves_pair_spin():
    g = model.gate(1.0, 0.37)
    for op in (model.SZ, model.SX):
        tot = np.kron(op, np.eye(3)) + np.kron(np.eye(3), op)
        assert np.abs(g @ tot - tot @ g).max() < 1e-14
    assert np.abs(g - g.T).max() < 1e-15


def test_swap_gate_exchanges_sites():
    rng = np.random.default_rng(0)
    a, b = rng.normal(size=3), rng.normal(size=3)
    assert np.allclose(model.swap_gate() @ np.kron(a, b), np.kron(b, a))


def test_spin1_algebra():
    # [S^+, S^-] = 2 S^z and S^2 = s(s+1) = 2 for spin one
    assert np.allclose(model.SP @ model.SM - model.SM @ model.SP,
                       2 * model.SZ)
    sy = (model.SP - model.SM) / 2j
    s2 = model.SX @ model.SX + sy @ sy + model.SZ @ model.SZ
    assert np.allclose(s2, 2 * np.eye(3))
    # S^x basis rows are orthonormal eigenvectors with eigenvalues +1,0,-1
    B = model.SX_BASIS
    assert np.allclose(B @ B.T, np.eye(3))
    assert np.allclose(B @ model.SX @ B.T, np.diag([1.0, 0.0, -1.0]))


# --------------------------------------------------------------------------
# exact references
# --------------------------------------------------------------------------
@pytest.mark.parametrize("beta", [0.5, 1.0, 2.0, 5.0])
def test_single_bond_closed_form(beta):
    # J (-2 e^{2bJ} - 3 e^{bJ} + 5 e^{-bJ}) / (e^{2bJ} + 3 e^{bJ} + 5 e^{-bJ})
    J = 1.0
    num = J * (-2 * math.exp(2 * beta * J) - 3 * math.exp(beta * J)
               + 5 * math.exp(-beta * J))
    den = (math.exp(2 * beta * J) + 3 * math.exp(beta * J)
           + 5 * math.exp(-beta * J))
    lat = model.chain(2)
    assert abs(exact.thermal_energy(lat, beta) - num / den) < 1e-13
    assert abs(exact.single_bond_energy(J, beta) - num / den) < 1e-13


def test_ed_high_temperature_series():
    lat = model.ladder(3, 1.0, 1.0)
    d1 = exact.thermal_energy(lat, 0.01) - exact.high_t_energy(lat, 0.01)
    d2 = exact.thermal_energy(lat, 0.005) - exact.high_t_energy(lat, 0.005)
    assert abs(d1) < 5e-6
    # the remainder is O(beta^3): halving beta divides it by about 8
    assert 6.0 < d1 / d2 < 10.0


def test_ed_ground_state_limit():
    lat = model.ladder(2, 1.0, 1.0)
    e0 = exact.ground_energy(lat)
    assert abs(exact.thermal_energy(lat, 60.0) - e0) < 1e-8


def test_trotter_error_is_second_order():
    lat = model.ladder(2, 1.0, 0.5)
    e = exact.thermal_energy(lat, 1.0)
    errs = [abs(exact.trotter_energy(lat, 1.0, t) - e)
            for t in (0.1, 0.05, 0.025)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5


def test_trotter_single_bond_is_exact():
    # one bond: the Trotter product of its own gate is e^{-beta h/2}
    lat = model.chain(2)
    assert abs(exact.trotter_energy(lat, 1.0, 0.1)
               - exact.single_bond_energy(1.0, 1.0)) < 1e-13


# --------------------------------------------------------------------------
# Philox
# --------------------------------------------------------------------------
@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)),
                                     ((7, 0), (3, 5, 11, 1)),
                                     ((2 ** 64 - 1, 12345),
                                      (2 ** 63, 1, 2 ** 64 - 2, 9))])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox increments the counter before every block, so its
    # first block for counter c is the published function at c + 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(ctr, dtype=np.uint64))
    raw = [int(x) for x in bg.random_raw(4)]
    c = list(ctr)
    c[0] = (c[0] + 1) % 2 ** 64
    if c[0] == 0:
        c[1] += 1
    assert list(philox.philox4x64(c, key)) == raw


def test_philox_uniform_range():
    us = [philox.uniform(3, c, 0, k, 0) for c in range(8) for k in range(64)]
    assert min(us) >= 0.0 and max(us) < 1.0
    assert abs(np.mean(us) - 0.5) < 0.05


# --------------------------------------------------------------------------
# layout and update list
# --------------------------------------------------------------------------
def test_layout_and_update_counts():
    # ladder 2x3 W=1 -> 8 MPS sites, 4 environment sites, 7 bonds, 25
    # updates per half-sweep (counted by hand from the snake order 0,1,3,2,4,5
    # with ancillas after sites 3 and 2)
    lat = model.ladder(3, 1.0, 1.0, W=1)
    lay = model.layout(lat)
    assert lay.length == 8
    assert lay.phys_of_pos == [0, 1, 3, -1, 2, -1, 4, 5]
    assert lay.env_positions == [0, 1, 6, 7]
    sch = model.schedule(lat, lay)
    assert [(p, q) for (p, q, _) in sch.mps_bonds] == [
        (0, 1), (0, 4), (1, 2), (2, 4), (2, 7), (4, 6), (6, 7)]
    assert len(sch.half) == 25 and len(sch.step) == 50
    for (L, W, n_up) in [(8, 2, 70), (16, 2, 126), (32, 4, 258)]:
        s = model.schedule(model.ladder(L, 1.0, 1.0, W=W))
        assert len(s.half) == n_up


def test_update_list_is_palindromic():
    sch = model.schedule(model.ladder(4, 1.0, 0.5, W=2))
    assert sch.step == sch.step[::-1]


def test_trotter_steps_integrality():
    assert model.trotter_steps(1.0, 0.1) == 5
    assert model.trotter_steps(5.0, 0.05) == 50
    assert model.trotter_steps(0.0, 0.05) == 0
    with pytest.raises(ValueError):
        model.trotter_steps(1.0, 0.3)


# --------------------------------------------------------------------------
# truncation rule
# --------------------------------------------------------------------------
def test_truncation_rank_cases():
    s = np.array([0.8, 0.5, 0.3, 1e-4, 1e-7])
    tot = float((s * s).sum())
    # cutoff just above the tail from index 3 keeps 3 values
    assert mps.truncation_rank(s, 10, (1e-8 + 1e-14) / tot * 1.01) == 3
    assert mps.truncation_rank(s, 10, 0.0) == 5
    assert mps.truncation_rank(s, 2, 0.0) == 2
    assert mps.truncation_rank(s, 10, 10.0) == 1          # never below one
    # a degenerate pair straddling the cap is dropped as a whole
    s2 = np.array([0.9, 0.3, 0.3, 0.3 * (1 - 1e-12), 0.01])
    assert mps.truncation_rank(s2, 2, 0.0) == 1
    assert mps.truncation_rank(s2, 3, 0.0) == 1
    assert mps.truncation_rank(s2, 4, 0.0) == 4
    # a run that starts at the top is kept as cut
    s3 = np.array([0.5, 0.5, 0.5, 0.5])
    assert mps.truncation_rank(s3, 2, 0.0) == 2


def test_truncation_tie_run_when_the_target_sets_the_cut():
    # Results section, third source of error: the discarded weight is held
    # at the target.  Spectrum with a three-fold run at indices 2..4; the
    # target alone would cut after index 2, inside the run.
    s = np.array([0.9, 0.3, 0.1, 0.1, 0.1 * (1 - 1e-12), 1e-3])
    tot = float((s * s).sum())            # 0.930001
    cut = 0.025 / tot                     # tail from 3 = 0.020001 < 0.025
    assert mps.truncation_rank(s, 100, cut) == 5   # the whole run is kept
    # discarded weight of that choice: only the last value, within target
    assert float((s[5:] ** 2).sum()) <= cut * tot
    # the run does not fit under the cap: the cap binds and the run is
    # dropped, even though the target alone would keep 3
    assert mps.truncation_rank(s, 4, cut) == 2
    assert mps.truncation_rank(s, 3, cut) == 2
    # exactly at the end of the run the cap admits it
    assert mps.truncation_rank(s, 5, cut) == 5
    # a target that cuts between runs is untouched by the tie rule
    assert mps.truncation_rank(s, 100, 0.05 / tot) == 2
    st = mps.Stats()
    mps.truncation_rank(s, 100, cut, st)
    assert st.ties == 1


def test_truncation_never_cuts_a_run_and_keeps_the_target_when_uncapped():
    # property over random spectra with planted runs of ties: with no
    # binding cap the discarded weight never exceeds the target, and no
    # cut (capped or not) falls between two tied values unless the run
    # starts at the largest value
    rng = np.random.default_rng(7)
    for trial in range(400):
        n = int(rng.integers(2, 40))
        s = np.sort(rng.exponential(size=n))[::-1].copy()
        for _ in range(int(rng.integers(0, 4))):
            i = int(rng.integers(0, n - 1))
            run = int(rng.integers(2, 5))
            s[i:i + run] = s[i] * (1 - 1e-12 * np.arange(run)[: n - i])
        s = np.sort(s)[::-1].copy()
        tot = float((s * s).sum())
        cut = float(10 ** rng.uniform(-6, -0.5))
        k = mps.truncation_rank(s, n, cut)
        assert 1 <= k <= n
        assert float((s[k:] ** 2).sum()) <= cut * tot * (1 + 1e-12)
        chi = int(rng.integers(1, n + 1))
        k2 = mps.truncation_rank(s, chi, cut)
        assert 1 <= k2 <= chi
        if k2 < n and s[k2 - 1] - s[k2] <= mps.TIE_TOL * s[k2 - 1]:
            # only a run that starts at sigma_0 may be cut
            assert np.all(s[0] - s[:k2 + 1] <= mps.TIE_TOL * s[0] * (k2 + 1))


# --------------------------------------------------------------------------
# whole MPS path against the dense Trotter product (exhaustive sums)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,W,basis", [(2, 0, 0), (2, 1, 1), (2, 2, 0),
                                       (3, 1, 0), (3, 1, 1)])
def test_exhaustive_hybrid_sum_equals_trotter(L, W, basis):
    lat = model.ladder(L, 1.0, 0.5 if L == 2 else 1.0, W=W)
    beta, tau = 1.0, 0.1
    ex = hybrid.exhaustive_average(lat, beta, tau, 10 ** 6, 0.0, basis)
    nb = len(lat.bonds)
    ops = [exact.hamiltonian(lat)] + [
        exact.bond_operator(i, j, lat.n_phys) for (i, j, _) in lat.bonds]
    ref = exact.trotter_average(lat, beta, tau, ops)
    assert abs(ex["energy"] - ref[0]) < 1e-12
    for b in range(nb):
        assert abs(ex["bond_ss"][b] - ref[1 + b]) < 1e-12


def test_ancilla_limit_single_bond_closed_form():
    # W = L on one rung: a single deterministic sample that is Trotter-exact
    lat = model.ladder(1, 1.0, 1.0, W=1)
    for beta in (0.5, 1.0, 2.0):
        ex = hybrid.exhaustive_average(lat, beta, 0.05, 100, 0.0)
        assert abs(ex["energy"] - exact.single_bond_energy(1.0, beta)) < 1e-12


def test_hybrid_sample_invariants():
    lat = model.ladder(3, 1.0, 1.0, W=1)
    lay = model.layout(lat)
    sch = model.schedule(lat, lay)
    env = {0: 0, 1: 2, 6: 1, 7: 0}          # m = +1, -1, 0, +1 -> M_E = 1
    psi, meas = hybrid.run_sample(lat, lay, sch, 5, 0.1, 10 ** 6, 0.0, env,
                                  0)
    assert abs(meas["norm"] - 1.0) < 1e-12
    assert abs(meas["qn"] - 1.0) < 1e-12
    # right-orthonormal sites after the centre returns to site 0
    for T in psi.tensors[1:]:
        l = T.shape[0]
        G = T.reshape(l, -1) @ T.reshape(l, -1).T
        assert np.abs(G - np.eye(l)).max() < 1e-12


def test_ancilla_limit_su2():
    # W = L: the state is SU(2) symmetric, <S^z_i> = 0 and zz = xx
    lat = model.ladder(2, 1.0, 0.5, W=2)
    lay = model.layout(lat)
    sch = model.schedule(lat, lay)
    psi, meas = hybrid.run_sample(lat, lay, sch, 10, 0.05, 10 ** 6, 0.0, {},
                                  0)
    L, R = mps._environments(psi.tensors)
    for p in range(lay.length):
        if lay.is_ancilla[p]:
            continue
        E = mps._transfer(L[p], psi.tensors[p], model.SZ)
        assert abs(np.sum(E * R[p])) < 1e-12
    p, q = lay.pos_of_phys[0], lay.pos_of_phys[2]
    vals = []
    for op in (model.SZ, model.SX):
        E = mps._transfer(L[p], psi.tensors[p], op)
        for m in range(p + 1, q):
            E = mps._transfer(E, psi.tensors[m])
        E = mps._transfer(E, psi.tensors[q], op)
        vals.append(float(np.sum(E * R[q])))
    assert abs(vals[0] - vals[1]) < 1e-12


def test_truncated_state_matches_untruncated_at_small_cutoff():
    lat = model.ladder(3, 1.0, 1.0, W=1)
    lay = model.layout(lat)
    sch = model.schedule(lat, lay)
    env = {0: 1, 1: 0, 6: 2, 7: 1}
    _, a = hybrid.run_sample(lat, lay, sch, 5, 0.1, 10 ** 6, 0.0, env, 0)
    st = mps.Stats()
    _, b = hybrid.run_sample(lat, lay, sch, 5, 0.1, 81, 1e-12, env, 0, st)
    assert st.max_chi <= 81
    # each update discards at most 1e-12 of the weight; the energy moves at
    # first order in the discarded amplitude: |dE| <~ |H| sqrt(sum eps)
    assert st.discarded <= 250 * 1e-12
    assert abs(a["energy"] - b["energy"]) < 20 * math.sqrt(st.discarded)
    # a binding cap of 32 discards a visible amount
    st32 = mps.Stats()
    hybrid.run_sample(lat, lay, sch, 5, 0.1, 32, 1e-12, env, 0, st32)
    assert st32.max_chi == 32 and st32.discarded > 1e-8


# --------------------------------------------------------------------------
# collapse: transition probabilities and detailed balance
# --------------------------------------------------------------------------
def _states(lay):
    for combo in itertools.product(range(3), repeat=len(lay.env_positions)):
        yield dict(zip(lay.env_positions, combo))


def test_beta_zero_collapse_table():
    lat = model.ladder(2, 1.0, 1.0, W=0)
    lay = model.layout(lat)
    sch = model.schedule(lat, lay)
    env = {0: 0, 1: 1, 2: 2, 3: 0}
    psi, _ = hybrid.run_sample(lat, lay, sch, 0, 0.05, 100, 0.0, env, 0)
    # same basis: the product state is returned with probability one
    assert abs(mps.outcome_probability(psi, lay, 0, env) - 1.0) < 1e-14
    # S^z -> S^x: |<x_t|e_s>|^2 rows (1/4,1/2,1/4), (1/2,0,1/2), (1/4,1/2,1/4)
    table = np.array([[0.25, 0.5, 0.25], [0.5, 0.0, 0.5], [0.25, 0.5, 0.25]])
    for j in _states(lay):
        expect = np.prod([table[env[p], j[p]] for p in lay.env_positions])
        assert abs(mps.outcome_probability(psi, lay, 1, j) - expect) < 1e-14


@pytest.mark.parametrize("basis", [0, 1])
def test_detailed_balance(basis):
    # P_i p(i -> j) is symmetric in i, j (Discussion of Detailed Balance)
    lat = model.ladder(2, 1.0, 0.5, W=1)
    lay = model.layout(lat)
    sch = model.schedule(lat, lay)
    states = list(_states(lay))
    P = np.zeros(len(states))
    T = np.zeros((len(states), len(states)))
    for a, i in enumerate(states):
        psi, meas = hybrid.run_sample(lat, lay, sch, 5, 0.1, 10 ** 6, 0.0, i,
                                      basis)
        P[a] = math.exp(meas["logw"])
        for b, j in enumerate(states):
            T[a, b] = mps.outcome_probability(psi, lay, basis, j)
    assert np.abs(T.sum(axis=1) - 1.0).max() < 1e-12
    F = P[:, None] * T
    assert np.abs(F - F.T).max() < 1e-12 * F.max()
    # stationarity: the weights P are a left eigenvector of the transitions
    assert np.abs(P @ T - P).max() < 1e-12 * P.max()


def test_collapse_frequencies_follow_probabilities():
    lat = model.ladder(2, 1.0, 1.0, W=1)
    lay = model.layout(lat)
    sch = model.schedule(lat, lay)
    env = dict(zip(lay.env_positions, (0, 2)))
    psi, _ = hybrid.run_sample(lat, lay, sch, 5, 0.1, 10 ** 6, 0.0, env, 0)
    states = list(_states(lay))
    probs = np.array([mps.outcome_probability(psi, lay, 1, j)
                      for j in states])
    counts = np.zeros(len(states))
    n = 1500
    index = {tuple(sorted(s.items())): a for a, s in enumerate(states)}
    for sample in range(n):
        import copy
        out = mps.collapse(copy.deepcopy(psi), lay, 1, 11, 0, sample)
        counts[index[tuple(sorted(out.items()))]] += 1
    exp = probs * n
    mask = exp > 5
    chi2 = float((((counts - exp) ** 2)[mask] / exp[mask]).sum())
    dof = int(mask.sum()) - 1
    # 99.9% quantile of chi^2 is below dof + 4 sqrt(2 dof) + 10 here
    assert chi2 < dof + 4 * math.sqrt(2 * dof) + 10


def test_z_only_chain_conserves_the_charge_within_each_sample():
    # every collapse in S^z: each evolution keeps Q = sum_phys S^z -
    # sum_anc S^z at the S^z total of its initial environment (the Bell
    # pairs carry Q = 0), the next sample starts in the sector of the
    # collapse outcomes, and that sector changes between samples
    # (Exploiting Conserved Quantum Numbers subsection).  The chain still
    # samples the thermal state: its mean agrees with ED.
    lat = model.ladder(3, 1.0, 1.0, W=1)
    recs = hybrid.run_chain(lat, 1.0, 0.1, 32, 1e-12, 24, seed=4,
                            z_only=True)
    charges = []
    for r in recs:
        assert r["basis"] == 0 and r["collapse_basis"] == 0
        q = sum(1 - r["env"][p] for p in r["env"])
        assert abs(r["qn"] - q) < 1e-10
        charges.append(q)
    for r0, r1 in zip(recs, recs[1:]):
        assert r1["env"] == r0["outcomes"]
    assert len(set(charges)) > 1
    mean, err = hybrid.estimate([r["energy"] for r in recs])
    assert abs(mean - exact.thermal_energy(lat, 1.0)) < 4 * err + 2e-4


def test_chain_mean_agrees_with_ed():
    # 2x3 ladder, W=1, beta=1, tau=0.1, chi_max=32, cutoff 1e-12, 20 samples
    lat = model.ladder(3, 1.0, 1.0, W=1)
    recs = hybrid.run_chain(lat, 1.0, 0.1, 32, 1e-12, 20, seed=0)
    mean, err = hybrid.estimate([r["energy"] for r in recs])
    e_ed = exact.thermal_energy(lat, 1.0)
    assert abs(mean - e_ed) < 4 * err + 2e-4
    for r in recs:
        assert abs(r["norm"] - 1.0) < 1e-10
        if r["basis"] == 0:
            me = sum(1 - r["env"][p] for p in r["env"])
            assert abs(r["qn"] - me) < 1e-10
