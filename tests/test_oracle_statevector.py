"""The oracle's MPS evolution against the same update list applied to the
full state vector over every MPS site (physical and ancilla), without
truncation (Ancilla Method subsection: two-site gates and swaps on an MPS;
Hybrid METTS-Ancilla subsection: the initial product state with Bell
pairs).  The vector is built here from its definition (unit S^z vectors
on environment sites, (1/sqrt 3) sum_s |s>|s> on each cluster site and its
ancilla) and evolved by 9 x 9 operators on neighbouring positions, so the
MPS machinery (contractions, SVD splits, absorb directions, centre moves)
is checked against plain linear algebra: the final vector to 1e-12 and the
log-weight (sum of ln ||G psi||^2 over the gates) to 1e-12."""
import math

import numpy as np
import pytest

from oracle import model, mps


def initial_vector(lay, outcomes):
    bell = np.eye(3).reshape(9) / math.sqrt(3.0)
    v = np.ones(1)
    p = 0
    while p < lay.length:
        if lay.is_cluster[p]:
            v = np.kron(v, bell)
            p += 2
        else:
            v = np.kron(v, np.eye(3)[outcomes[p]])
            p += 1
    return v


def apply_two_site(v, op, k, n):
    t = v.reshape(3 ** k, 9, 3 ** (n - k - 2))
    return np.einsum("uv,avb->aub", op, t).reshape(-1)


def mps_vector(psi):
    v = psi.tensors[0]
    for T in psi.tensors[1:]:
        v = np.tensordot(v, T, axes=([v.ndim - 1], [0]))
    return v.reshape(-1)


@pytest.mark.parametrize("L, W, labels", [
    (3, 1, (0, 1, 2, 1)),        # 2x3 ladder, one purified column
    (3, 0, (2, 0, 1, 0, 2, 1)),  # no cluster: METTS
    (2, 2, ()),                  # every column purified: ancilla limit
])
def test_untruncated_evolution_equals_state_vector(L, W, labels):
    beta, tau = 0.6, 0.1
    lat = model.ladder(L, 1.0, 0.7, W=W)
    lay = model.layout(lat)
    sch = model.schedule(lat, lay)
    M = model.trotter_steps(beta, tau)
    outcomes = dict(zip(lay.env_positions, labels))
    n = lay.length
    v = initial_vector(lay, outcomes)
    logw = 0.0
    swap = model.swap_gate()
    gates = [model.gate(J, tau / 2.0) for J in sch.couplings]
    for u in model.evolve_updates(sch, M):
        if u.op == model.OP_SWAP:
            v = apply_two_site(v, swap, u.k, n)
        else:
            v = apply_two_site(v, gates[u.op], u.k, n)
            n2 = float(v @ v)
            logw += math.log(n2)
            v /= math.sqrt(n2)
    psi = mps.init_state(lay, outcomes, 0)
    mps.evolve(psi, sch, M, tau, 3 ** (n // 2), 0.0)
    got = mps_vector(psi)
    assert abs(np.linalg.norm(got) - 1.0) < 1e-13
    assert np.abs(got - v).max() < 1e-12
    assert abs(psi.logw - logw) < 1e-12
