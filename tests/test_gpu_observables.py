"""Long-range observables on the GPU (through the C ABI) against the FP64
oracle: correlators of arbitrary spin pairs and the susceptibility
estimator chi_6 (Results section), and the per-bond sample moments of the
variance study (Entanglement and Cost of Hybrid States).  Tolerances:
1e-10 absolute on correlators and on the moments, 1e-10 relative on chi;
the exhaustive identity 1e-11."""
import itertools

import numpy as np
import pytest

from oracle import exact, hybrid, model, mps, observables
from paper_1910_09142_amd import hmps, workloads
from test_oracle_observables import spin_total_squared

pytestmark = pytest.mark.gpu


def gpu_state(L, W, beta, tau, chi, cut, states=None, seed=0, basis=0,
              n_chains=None):
    n, bonds, order, mask = workloads.ladder_arrays(L, 1.0, 1.0, W)
    lat = hmps.Lattice(n, bonds, order, mask)
    B = len(states) if states is not None else (n_chains or 1)
    ctx = hmps.Context(B, workloads.mps_length(L, W), chi, len(bonds))
    ctx.hmps_init_cluster_env(lat, B, seed, env_state=states, basis=basis)
    ctx.hmps_evolve(beta, tau, chi, cut)
    return ctx


def oracle_state(L, W, beta, tau, chi, cut, env, basis=0):
    olat = model.ladder(L, 1.0, 1.0, W=W)
    lay = model.layout(olat)
    psi = mps.init_state(lay, env, basis)
    mps.evolve(psi, model.schedule(olat, lay), model.trotter_steps(beta, tau),
               tau, chi, cut)
    return psi, olat, lay


def test_pair_correlators_against_oracle():
    # 2x4 ladder, W=2; every ordered pair (self pairs included), repeated
    # so that the list spans several passes of the device
    L, W, beta, tau, chi, cut = 4, 2, 1.0, 0.1, 64, 1e-12
    states = np.array([[0, 1, 2, 0], [2, 2, 1, 1], [1, 0, 0, 2]], np.uint8)
    pairs = [(i, j) for i in range(8) for j in range(8)] * 5
    print("case: pair correlators 2x4", flush=True)
    ctx = gpu_state(L, W, beta, tau, chi, cut, states=states)
    g = ctx.hmps_measure_pairs(pairs)
    ctx.hmps_destroy()
    for c in range(len(states)):
        olat = model.ladder(L, 1.0, 1.0, W=W)
        lay = model.layout(olat)
        env = dict(zip(lay.env_positions, states[c].tolist()))
        psi, olat, lay = oracle_state(L, W, beta, tau, chi, cut, env)
        r = np.array(observables.pair_correlations(psi, olat, lay, pairs))
        print(f"  chain {c}: max |d| {np.abs(g[c] - r).max():.2e}", flush=True)
        assert np.abs(g[c] - r).max() <= 1e-10


def test_chi6_against_oracle():
    # 2x8 ladder, W=2, beta=0.5: chi over the middle 6x2 sites
    L, W, beta, tau, chi, cut, seed = 8, 2, 0.5, 0.05, 128, 1e-12, 0
    center = workloads.central_sites(L)
    print("case: chi_6 on 2x8", flush=True)
    ctx = gpu_state(L, W, beta, tau, chi, cut, seed=seed)
    g = ctx.hmps_susceptibility(beta, center)[0]
    ctx.hmps_destroy()
    olat = model.ladder(L, 1.0, 1.0, W=W)
    lay = model.layout(olat)
    env = mps.initial_outcomes(lay, seed, 0)
    psi, olat, lay = oracle_state(L, W, beta, tau, chi, cut, env)
    r = observables.susceptibility(psi, olat, lay, beta, center)
    print(f"  chi_6 gpu={g:.15f} oracle={r:.15f}", flush=True)
    assert abs(g - r) <= 1e-10 * abs(r)


@pytest.mark.parametrize("basis", [0, 1])
def test_exhaustive_susceptibility_equals_dense(basis):
    L, W, beta, tau = 2, 1, 1.0, 0.1
    olat = model.ladder(L, 1.0, 1.0, W=W)
    lay = model.layout(olat)
    states = np.array(list(itertools.product(range(3),
                                             repeat=len(lay.env_positions))),
                      np.uint8)
    print(f"case: exhaustive chi basis {basis}", flush=True)
    ctx = gpu_state(L, W, beta, tau, 81, 0.0, states=states, basis=basis)
    chi = ctx.hmps_susceptibility(beta, list(range(olat.n_phys)))
    logw = ctx.hmps_measure()["logw"]
    ctx.hmps_destroy()
    w = np.exp(logw - logw.max())
    avg = float((w * chi).sum() / w.sum())
    X = spin_total_squared(olat)
    ref = beta / 3.0 * exact.trotter_average(olat, beta, tau, [X])[0] / olat.n_phys
    print(f"  chi gpu {avg:.14f} dense {ref:.14f}", flush=True)
    assert abs(avg - ref) < 1e-11


def test_bond_moments_against_oracle_chains():
    # 2x3 ladder (W = 1, beta = 1, tau = 0.1, chi_max = 32, cutoff 1e-12):
    # four chains, eight samples each, their outcomes bit-exact with the
    # oracle's (no draw near a threshold); the device accumulates the
    # per-bond moments, the oracle takes the definition over the same 32
    # samples
    L, W, beta, tau, chi, cut, N, C = 3, 1, 1.0, 0.1, 32, 1e-12, 8, 4
    print(f"case: bond moments, 2x{L} ladder, {C} chains x {N} samples",
          flush=True)
    n, bonds, order, mask = workloads.ladder_arrays(L, 1.0, 1.0, W)
    lat = hmps.Lattice(n, bonds, order, mask)
    ctx = hmps.Context(C, workloads.mps_length(L, W), chi, len(bonds))
    ctx.hmps_init_cluster_env(lat, C, 0)
    for k in range(N):
        ctx.hmps_evolve(beta, tau, chi, cut)
        ctx.hmps_measure(hmps.MEASURE_ACCUMULATE)
        ctx.hmps_collapse_resample(k % 2)
    got = ctx.hmps_bond_moments()
    olat = model.ladder(L, 1.0, 1.0, W=W)
    rows, energies = [], []
    for c in range(C):
        for r in hybrid.run_chain(olat, beta, tau, chi, cut, N, seed=0,
                                  chain=c):
            assert r["near"] == 0
            rows.append(r["bond_ss"])
            energies.append([r["energy"]])
    n_ref, mean, var = observables.sample_moments(rows)
    _, emean, evar = observables.sample_moments(energies)
    print(f"  var gpu {np.round(got['var'], 6).tolist()}", flush=True)
    assert got["n"] == n_ref == C * N
    assert np.abs(got["mean"] - np.array(mean)).max() < 1e-10
    assert np.abs(got["var"] - np.array(var)).max() < 1e-10
    assert abs(got["energy_mean"] - emean[0]) < 1e-10 * abs(emean[0])
    assert abs(got["energy_var"] - evar[0]) < 1e-10
    # a reset clears the moments: with none accumulated there is no
    # variance (E_STATE); one measurement then gives one value per chain
    ctx.hmps_moments_reset()
    with pytest.raises(hmps.HmpsError) as e:
        ctx.hmps_bond_moments()
    assert e.value.status == hmps.HMPS_E_STATE
    m = ctx.hmps_measure(hmps.MEASURE_BONDS | hmps.MEASURE_ACCUMULATE)
    got = ctx.hmps_bond_moments()
    _, mean, var = observables.sample_moments(m["bond_ss"])
    assert got["n"] == C
    assert np.abs(got["mean"] - np.array(mean)).max() < 1e-14
    assert np.abs(got["var"] - np.array(var)).max() < 1e-14
    ctx.hmps_destroy()
