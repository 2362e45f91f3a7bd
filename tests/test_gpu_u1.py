"""U(1)-symmetric evolution (HMPS_SYM_U1) through the C ABI.

The hybrid method collapses only the environment, in S^z: every evolution
then conserves Q = sum_phys S^z - sum_anc S^z (Bell pairs carry Q = 0 with
the ancilla counted with flipped sign), its tensors are block sparse, and Q
still changes from sample to sample (Exploiting Conserved Quantum Numbers
subsection).  The library splits each update's theta' into its charge
blocks, decomposes them separately, and truncates their singular values
together.

Reference: the dense FP64 oracle with every collapse in S^z
(hybrid.run_chain(z_only=True)); the block-sparse SVD is exact, so the
tolerances are those of the dense parity tests (energy 1e-10 relative,
<S_i.S_j> 1e-10, log-weight 1e-9, <Q> 1e-10, collapse outcomes bit-exact).
Also checked: the untruncated exhaustive batch against the Trotter thermal
average (1e-11); the charges the library reports against the nonzero
pattern of every site tensor (exactly zero outside the blocks); <Q> equal
to the charge of the last bond; the dense GPU path on the 2x8 ladder at
the cap and on the 2x16 ladder at chi_max = 256; and results independent of
how the blocks are grouped in passes.
"""
import itertools

import numpy as np
import pytest

from oracle import exact, hybrid, model, mps
from paper_1910_09142_amd import hmps, workloads

pytestmark = pytest.mark.gpu

TIGHT = {"e_rel": 1e-10, "ss": 1e-10, "logw": 1e-9, "qn": 1e-10}


def u1_ctx(L, W, chi_cap, n_chains, max_blocks=0, symmetry=hmps.SYM_U1):
    n, bonds, order, mask = workloads.ladder_arrays(L, 1.0, 1.0, W)
    lat = hmps.Lattice(n, bonds, order, mask)
    ctx = hmps.Context(n_chains, workloads.mps_length(L, W), chi_cap,
                       len(bonds), symmetry=symmetry, max_blocks=max_blocks)
    return ctx, lat


def run_u1_chain(L, W, beta, tau, chi, cut, n_samples, seed, n_chains=1,
                 max_blocks=0, symmetry=hmps.SYM_U1):
    ctx, lat = u1_ctx(L, W, chi, n_chains, max_blocks, symmetry)
    ctx.hmps_init_cluster_env(lat, n_chains, seed)
    out = []
    for _ in range(n_samples):
        ctx.hmps_evolve(beta, tau, chi, cut)
        m = ctx.hmps_measure()
        m["outcomes"] = ctx.hmps_collapse_resample(0)
        out.append(m)
    blocks = ctx.hmps_stats().u1_blocks
    ctx.hmps_destroy()
    return out, blocks


def test_u1_chain_matches_the_oracle():
    # 2x3 ladder, W=1, beta=1, tau=0.1, chi_max=32, cutoff 1e-12, seed 0,
    # every collapse in S^z
    L, W, beta, tau, chi, cut, N = 3, 1, 1.0, 0.1, 32, 1e-12, 12
    print("case: U(1) C1 chain, 12 samples", flush=True)
    gpu, blocks = run_u1_chain(L, W, beta, tau, chi, cut, N, 0)
    assert blocks > 0
    olat = model.ladder(L, 1.0, 1.0, W=W)
    ref = hybrid.run_chain(olat, beta, tau, chi, cut, N, seed=0, z_only=True)
    lay = model.layout(olat)
    charges = set()
    for n in range(N):
        g, r = gpu[n], ref[n]
        e = r["energy"]
        print(f"  sample {n}: E gpu={g['energy'][0]:.15f} oracle={e:.15f} "
              f"Q={g['qn'][0]:.12f}", flush=True)
        assert abs(g["energy"][0] - e) <= TIGHT["e_rel"] * abs(e)
        assert np.abs(g["bond_ss"][0] - np.array(r["bond_ss"])).max() <= \
            TIGHT["ss"]
        assert abs(g["logw"][0] - r["logw"]) <= TIGHT["logw"]
        q = sum(1 - v for v in r["env"].values())
        assert abs(g["qn"][0] - q) <= TIGHT["qn"]
        charges.add(q)
        want = [r["outcomes"][p] for p in lay.env_positions]
        got = list(g["outcomes"][0])
        if got != want:
            assert r["near"] > 0, f"sample {n}: {got} != {want}"
            break
    # the sector moves between samples (the paper's histogram of Q)
    assert len(charges) > 1


def test_u1_exhaustive_batch_equals_trotter():
    # all 81 S^z environment states of the 2x3 W=1 ladder, untruncated: the
    # P-weighted mean is the Trotter thermal average.  81 chains with up to
    # 9 blocks each in passes of at most 200 blocks: the updates run in
    # several passes.
    L, W, beta, tau = 3, 1, 1.0, 0.1
    olat = model.ladder(L, 1.0, 1.0, W=W)
    states = np.array(list(itertools.product(range(3), repeat=4)), np.uint8)
    print("case: U(1) exhaustive batch", flush=True)
    ctx, lat = u1_ctx(L, W, 81, len(states), max_blocks=200)
    ctx.hmps_init_cluster_env(lat, len(states), 0, env_state=states)
    ctx.hmps_evolve(beta, tau, 81, 0.0)
    g = ctx.hmps_measure()
    ctx.hmps_destroy()
    w = np.exp(g["logw"] - g["logw"].max())
    avg = float((w * g["energy"]).sum() / w.sum())
    ref = exact.trotter_energy(olat, beta, tau)
    print(f"  weighted mean {avg:.15f} Trotter {ref:.15f}", flush=True)
    assert abs(avg - ref) < 1e-11
    # Q of each chain is its environment's S^z total
    q = (1 - states.astype(int)).sum(axis=1)
    assert np.abs(g["qn"] - q).max() < 1e-10


def check_charges(ctx, lat_layout, n_chains):
    """Every site tensor vanishes outside its charge blocks; <Q> is the
    charge of the last bond."""
    chi = ctx.hmps_bond_dims()
    n_sites = chi.shape[1] - 1
    is_anc = lat_layout.is_ancilla
    m = ctx.hmps_measure()
    for c in range(n_chains):
        q = [ctx.hmps_bond_charges(c, b) for b in range(n_sites + 1)]
        assert q[0].tolist() == [0]
        assert abs(m["qn"][c] - q[n_sites][0]) < 1e-10
        for p in range(n_sites):
            T = ctx.hmps_read_site(c, p)
            sign = -1 if is_anc[p] else 1
            sz = 1 - np.arange(3)
            allowed = (q[p + 1][None, None, :] ==
                       q[p][None, :, None] + sign * sz[:, None, None])
            assert np.abs(T[~allowed]).max(initial=0.0) == 0.0, (c, p)
            # every index of the bond is used by the block it is in
            assert np.abs(T).max() > 0.0


def test_u1_charges_label_the_site_tensors():
    # 2x8 ladder, W=2, chi_max=64, five Trotter steps (beta 0.5, tau 0.05)
    L, W = 8, 2
    print("case: U(1) charges, 2x8 W=2", flush=True)
    ctx, lat = u1_ctx(L, W, 64, 3)
    ctx.hmps_init_cluster_env(lat, 3, 11)
    ctx.hmps_evolve(0.5, 0.05, 64, 1e-12)
    lay = model.layout(model.ladder(L, 1.0, 1.0, W=W))
    check_charges(ctx, lay, 3)
    ctx.hmps_collapse_resample(0)
    check_charges(ctx, lay, 3)
    ctx.hmps_destroy()


def test_u1_matches_the_dense_path_at_the_cap():
    # 2x8 ladder, W=2, beta=1, tau=0.05, chi_max=128 (the cap binds), 4
    # chains, two samples: the dense and the block-sparse path agree to the
    # level at which a capped sample depends on the last bits of each SVD
    L, W, beta, tau, chi, cut = 8, 2, 1.0, 0.05, 128, 1e-12
    print("case: U(1) vs dense, 2x8 at chi 128", flush=True)
    u1, blocks = run_u1_chain(L, W, beta, tau, chi, cut, 2, 3, n_chains=4)
    dense, _ = run_u1_chain(L, W, beta, tau, chi, cut, 2, 3, n_chains=4,
                            symmetry=hmps.SYM_NONE)
    assert blocks > 0
    for n in range(2):
        g, d = u1[n], dense[n]
        de = np.abs(g["energy"] - d["energy"]) / np.abs(d["energy"])
        print(f"  sample {n}: max dE/E {de.max():.2e}", flush=True)
        assert de.max() <= 1e-8
        assert np.abs(g["bond_ss"] - d["bond_ss"]).max() <= 2.5e-7
        assert np.abs(g["logw"] - d["logw"]).max() <= 1e-6
        assert np.abs(g["qn"] - np.round(g["qn"])).max() <= 1e-10
        assert np.array_equal(g["outcomes"], d["outcomes"])


def test_u1_matches_the_dense_path_on_the_2x16_ladder():
    # 2x16 ladder, W=2, J_rung=0.5, tau=0.05, chi_max=256, cutoff 1e-10,
    # 8 chains, the first 6 Trotter steps (bonds reach chi ~ 200, theta' up
    # to 768 x 768 split into its charge blocks): energies and correlators
    # of the two paths agree at the level of a capped free-running state
    wl = workloads.C3
    L, W = wl.L, wl.W
    print("case: U(1) vs dense, 2x16 at chi 256, 6 steps", flush=True)
    n, bonds, order, mask = workloads.ladder_arrays(L, wl.J_leg, wl.J_rung,
                                                    W)
    lat = hmps.Lattice(n, bonds, order, mask)
    out = {}
    for sym in (hmps.SYM_U1, hmps.SYM_NONE):
        ctx = hmps.Context(8, workloads.mps_length(L, W), wl.chi_max,
                           len(bonds), symmetry=sym)
        ctx.hmps_init_cluster_env(lat, 8, 17)
        ctx.hmps_evolve(0.6, wl.tau, wl.chi_max, wl.cutoff)
        out[sym] = (ctx.hmps_measure(), ctx.hmps_bond_dims(),
                    ctx.hmps_stats().u1_blocks)
        ctx.hmps_destroy()
    (gu, chiu, blocks), (gd, chid, _) = out[hmps.SYM_U1], out[hmps.SYM_NONE]
    assert blocks > 0
    de = np.abs(gu["energy"] - gd["energy"]) / np.abs(gd["energy"])
    print(f"  max dE/E {de.max():.2e}, max chi {chiu.max()}", flush=True)
    assert chiu.max() > 128
    assert de.max() <= 1e-8
    assert np.abs(gu["bond_ss"] - gd["bond_ss"]).max() <= 2.5e-7
    assert np.abs(gu["logw"] - gd["logw"]).max() <= 1e-6
    assert np.abs(gu["qn"] - np.round(gu["qn"])).max() <= 1e-10


def test_u1_results_do_not_depend_on_the_passes():
    # the blocks of an update (up to 9 per chain, 3 chains) split over
    # passes of at most 12 blocks give the same bits as one pass
    L, W, beta, tau, chi, cut = 3, 1, 1.0, 0.1, 32, 1e-12
    print("case: U(1) passes", flush=True)
    one, _ = run_u1_chain(L, W, beta, tau, chi, cut, 2, 5, n_chains=3)
    many, _ = run_u1_chain(L, W, beta, tau, chi, cut, 2, 5, n_chains=3,
                           max_blocks=12)
    for a, b in zip(one, many):
        for key in ("energy", "bond_ss", "logw", "qn", "outcomes"):
            assert np.array_equal(a[key], b[key]), key


def test_u1_rejects_what_breaks_the_symmetry():
    L, W = 3, 1
    ctx, lat = u1_ctx(L, W, 16, 2)
    states = np.zeros((2, 4), np.uint8)
    with pytest.raises(hmps.HmpsError, match="status 1"):
        ctx.hmps_init_cluster_env(lat, 2, 0, env_state=states, basis=1)
    ctx.hmps_init_cluster_env(lat, 2, 0)
    ctx.hmps_evolve(0.2, 0.1, 16, 1e-12)
    with pytest.raises(hmps.HmpsError, match="status 1"):
        ctx.hmps_collapse_resample(1)
    ctx.hmps_collapse_resample(0)
    # a chain with more blocks than max_blocks: E_NOMEM before any launch
    small, lat2 = u1_ctx(L, W, 16, 1, max_blocks=1)
    small.hmps_init_cluster_env(lat2, 1, 0)
    with pytest.raises(hmps.HmpsError, match="status 2"):
        small.hmps_evolve(0.2, 0.1, 16, 1e-12)
    small.hmps_destroy()
    # charges exist only for chains of a U(1) context's own initialisation
    center, right = workloads.bond_tensors(0, 1, 4, 4, 4)
    ctx.hmps_load_bond(center, right)
    with pytest.raises(hmps.HmpsError, match="status 4"):
        ctx.hmps_bond_charges(0, 1)
    ctx.hmps_destroy()
    dense, lat3 = u1_ctx(L, W, 16, 1, symmetry=hmps.SYM_NONE)
    dense.hmps_init_cluster_env(lat3, 1, 0)
    with pytest.raises(hmps.HmpsError, match="status 4"):
        dense.hmps_bond_charges(0, 1)
    dense.hmps_destroy()
    with pytest.raises(hmps.HmpsError, match="status 1"):
        hmps.Context(1, 6, 16, 7, precision=hmps.PREC_MIXED_FP32,
                     symmetry=hmps.SYM_U1)
