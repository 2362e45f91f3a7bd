"""Pins of the oracle's long-range observables (pair correlators and the
susceptibility estimator) against dense exact diagonalisation and product
states."""
import itertools

import numpy as np
import pytest

from oracle import exact, model, mps, observables


def spin_total_squared(lat, center=None):
    """Dense sum_{j in C} sum_i S_j.S_i (C = all sites: S_tot^2)."""
    n = lat.n_phys
    center = range(n) if center is None else center
    pairs = [(j, i, 1.0) for j in center for i in range(n) if i != j]
    pseudo = model.Lattice(n, pairs, lat.order, lat.in_cluster)
    dim = 3 ** n
    return exact.hamiltonian(pseudo) + 2.0 * len(list(center)) * np.eye(dim)


@pytest.mark.parametrize("basis", [0, 1])
@pytest.mark.parametrize("center", [None, (1, 2)])
def test_exhaustive_susceptibility_equals_dense(basis, center):
    # 2x2 ladder, one purified column: the P-weighted mean of the sample
    # estimator over all environment states equals the dense Trotter
    # average (beta/3)(1/|C|) Tr[X U^2]/Tr[U^2], X = sum_{j in C} sum_i S_j.S_i
    L, W, beta, tau = 2, 1, 1.0, 0.1
    lat = model.ladder(L, 1.0, 1.0, W=W)
    lay = model.layout(lat)
    sch = model.schedule(lat, lay)
    M = model.trotter_steps(beta, tau)
    C = list(range(lat.n_phys)) if center is None else list(center)
    num = den = 0.0
    for labels in itertools.product(range(3), repeat=len(lay.env_positions)):
        psi = mps.init_state(lay, dict(zip(lay.env_positions, labels)), basis)
        mps.evolve(psi, sch, M, tau, 81, 0.0)
        w = np.exp(psi.logw)
        num += w * observables.susceptibility(psi, lat, lay, beta, C)
        den += w
    X = spin_total_squared(lat, C)
    ref = beta / 3.0 * exact.trotter_average(lat, beta, tau, [X])[0] / len(C)
    assert abs(num / den - ref) < 1e-12


def test_product_state_correlators():
    # no evolution (beta = 0, no cluster): <S_i.S_j> = m_i m_j for i != j
    lat = model.ladder(3, 1.0, 1.0, W=0)
    lay = model.layout(lat)
    labels = [0, 2, 1, 0, 2, 2]          # m = +1, -1, 0, +1, -1, -1
    env = dict(zip(lay.env_positions, labels))
    psi = mps.init_state(lay, env, 0)
    m = {lay.phys_of_pos[p]: 1 - s for p, s in env.items()}
    pairs = [(i, j) for i in range(6) for j in range(6)]
    vals = observables.pair_correlations(psi, lat, lay, pairs)
    for (i, j), v in zip(pairs, vals):
        want = 2.0 if i == j else m[i] * m[j]
        assert abs(v - want) < 1e-14


def test_sample_moments_closed_forms():
    # a hand-computed sample: 1, 2, 3, 4 -> mean 5/2, variance 5/3
    n, mean, var = observables.sample_moments([[1.0], [2.0], [3.0], [4.0]])
    assert n == 4 and mean == [2.5] and abs(var[0] - 5.0 / 3.0) < 1e-15
    # a constant column has zero variance; columns are independent
    n, mean, var = observables.sample_moments([[0.3, -1.0], [0.3, 1.0]] * 3)
    assert mean == pytest.approx([0.3, 0.0]) and var[0] == 0.0
    # two values a, b with counts k and n - k: variance k (n - k) (a - b)^2
    # / (n (n - 1)), mean (k a + (n - k) b) / n
    a, b, k, n = -0.75, 0.25, 7, 19
    rows = [[a]] * k + [[b]] * (n - k)
    got_n, mean, var = observables.sample_moments(rows)
    assert got_n == n
    assert abs(mean[0] - (k * a + (n - k) * b) / n) < 1e-15
    assert abs(var[0] - k * (n - k) * (a - b) ** 2 / (n * (n - 1))) < 1e-15
    with pytest.raises(ValueError):
        observables.sample_moments([[1.0]])
