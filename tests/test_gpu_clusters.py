"""Clusters that are not contiguous: any set of physical sites can be
purified by ancilla partners while the rest is sampled (the partition is an
input of the method; the conclusion suggests interleaving purified and
sampled sites).  The exhaustive identity sum_i P_i <A>_i / sum_i P_i =
Tr[A U^2] / Tr[U^2] holds for every partition, and single chains follow the
oracle sample by sample (outcomes bit-exact)."""
import itertools

import numpy as np
import pytest

from oracle import exact, hybrid, model
from paper_1910_09142_amd import hmps, workloads
from test_gpu_parity import compare_sample

pytestmark = pytest.mark.gpu


def masked_ladder(L, cluster_sites, J_rung=1.0):
    base = model.ladder(L, 1.0, J_rung, W=0)
    in_cluster = [i in cluster_sites for i in range(base.n_phys)]
    olat = model.Lattice(base.n_phys, base.bonds, base.order, in_cluster,
                         name=f"ladder{L}x2_sites{sorted(cluster_sites)}")
    glat = hmps.Lattice(base.n_phys, base.bonds, base.order,
                        [int(x) for x in in_cluster])
    return olat, glat


def gpu_context(olat, n_chains, chi):
    n_sites = olat.n_phys + sum(olat.in_cluster)
    return hmps.Context(n_chains, n_sites, chi, len(olat.bonds))


def test_checkerboard_cluster_exhaustive_equals_trotter():
    # 2x3 ladder, cluster = sites 0, 3, 4 (alternating legs), untruncated
    L, beta, tau = 3, 1.0, 0.1
    olat, glat = masked_ladder(L, {0, 3, 4})
    lay = model.layout(olat)
    n_env = len(lay.env_positions)
    states = np.array(list(itertools.product(range(3), repeat=n_env)),
                      np.uint8)
    ref = exact.trotter_energy(olat, beta, tau)
    for basis in (0, 1):
        print(f"case: checkerboard cluster, basis {basis}", flush=True)
        ctx = gpu_context(olat, len(states), 81)
        ctx.hmps_init_cluster_env(glat, len(states), 0, env_state=states,
                                  basis=basis)
        ctx.hmps_evolve(beta, tau, 81, 0.0)
        g = ctx.hmps_measure()
        ctx.hmps_destroy()
        w = np.exp(g["logw"] - g["logw"].max())
        avg = float((w * g["energy"]).sum() / w.sum())
        print(f"  weighted mean {avg:.13f} Trotter {ref:.13f}", flush=True)
        assert abs(avg - ref) < 1e-11


def test_interleaved_columns_chain():
    # 2x4 ladder, cluster = columns 0 and 2, three samples of one chain
    L, beta, tau, chi, cut, N, seed = 4, 1.0, 0.1, 32, 1e-12, 3, 2
    olat, glat = masked_ladder(L, {0, 1, 4, 5})
    lay = model.layout(olat)
    print("case: interleaved columns chain", flush=True)
    ctx = gpu_context(olat, 1, chi)
    ctx.hmps_init_cluster_env(glat, 1, seed)
    gpu = []
    for n in range(N):
        ctx.hmps_evolve(beta, tau, chi, cut)
        m = ctx.hmps_measure()
        m["outcomes"] = ctx.hmps_collapse_resample(n % 2)
        gpu.append(m)
    ctx.hmps_destroy()
    ref = hybrid.run_chain(olat, beta, tau, chi, cut, N, seed=seed)
    for n in range(N):
        compare_sample(gpu[n], ref[n])
        want = [ref[n]["outcomes"][p] for p in lay.env_positions]
        got = list(gpu[n]["outcomes"][0])
        if got != want:
            assert ref[n]["near"] > 0, f"sample {n}: {got} != {want}"
            break


def test_checkerboard_cluster_u1():
    # the checkerboard cluster with U(1) updates: ancillas sit between
    # physical sites of the MPS and swaps move them past the sampled sites,
    # so the charge of every position follows the swaps.  The exhaustive
    # S^z batch equals the Trotter average, every chain's <Q> is its
    # environment's S^z total, and the site tensors vanish outside their
    # charge blocks.
    L, beta, tau = 3, 1.0, 0.1
    olat, glat = masked_ladder(L, {0, 3, 4})
    lay = model.layout(olat)
    n_env = len(lay.env_positions)
    states = np.array(list(itertools.product(range(3), repeat=n_env)),
                      np.uint8)
    print("case: checkerboard cluster, U(1)", flush=True)
    n_sites = olat.n_phys + sum(olat.in_cluster)
    ctx = hmps.Context(len(states), n_sites, 81, len(olat.bonds),
                       symmetry=hmps.SYM_U1)
    ctx.hmps_init_cluster_env(glat, len(states), 0, env_state=states)
    ctx.hmps_evolve(beta, tau, 81, 0.0)
    g = ctx.hmps_measure()
    w = np.exp(g["logw"] - g["logw"].max())
    avg = float((w * g["energy"]).sum() / w.sum())
    ref = exact.trotter_energy(olat, beta, tau)
    print(f"  weighted mean {avg:.13f} Trotter {ref:.13f}", flush=True)
    assert abs(avg - ref) < 1e-11
    q = (1 - states.astype(int)).sum(axis=1)
    assert np.abs(g["qn"] - q).max() < 1e-10
    sz = 1 - np.arange(3)
    for c in (0, 13, len(states) - 1):
        qs = [ctx.hmps_bond_charges(c, b) for b in range(n_sites + 1)]
        for p in range(n_sites):
            T = ctx.hmps_read_site(c, p)
            sign = -1 if lay.is_ancilla[p] else 1
            allowed = (qs[p + 1][None, None, :] ==
                       qs[p][None, :, None] + sign * sz[:, None, None])
            assert np.abs(T[~allowed]).max(initial=0.0) == 0.0, (c, p)
    ctx.hmps_destroy()
