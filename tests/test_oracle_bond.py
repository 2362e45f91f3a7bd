"""The synthetic bond of the single-gate workload and the oracle's two-site
update on it, pinned by facts that do not come from the oracle:

* the generator: B right-orthonormal, the centre's Schmidt values on its
  right bond equal to the prescribed exp(-j/decay) profile (unit norm);
* with the identity gate and no truncation the update returns exactly
  those Schmidt values (for a right-orthonormal B the Schmidt values of
  C B are those of C), keeps the state and adds ln 1 = 0 to the log-weight;
* G_J(x) followed by G_J(-x) without truncation restores the state (the
  two exponentials are inverse), and the two log-weight increments add up
  to ln ||G theta||^2 + ln ||G^-1 G theta / ||G theta||||^2 = 0;
* the total spin of the pair is conserved: G commutes with S_1.S_2, so
  <S_1.S_2> of the two physical indices is unchanged by an untruncated
  gate (after renormalisation it changes only through the weights of the
  spin sectors, which the closed form below predicts).
"""
import math

import numpy as np
import pytest

from oracle import model, mps
from paper_1910_09142_amd import workloads


def to_oracle(T):
    return np.ascontiguousarray(T.transpose(1, 0, 2))


def two_site(psi):
    A, B = psi.tensors
    return np.einsum("asb,btc->astc", A, B)


@pytest.mark.parametrize("dims", [(4, 10, 5), (16, 16, 16), (7, 20, 9)])
def test_generator_profile(dims):
    l, m, r = dims
    center, right = workloads.bond_tensors(1, 2, l, m, r, decay=6.0)
    want = np.exp(-np.arange(m) / 6.0)
    want /= np.linalg.norm(want)
    for c in range(2):
        B = right[c]
        assert np.abs(np.einsum("sbc,sdc->bd", B, B) - np.eye(m)).max() < 1e-13
        cm = center[c].transpose(1, 0, 2).reshape(3 * l, m)
        s = np.linalg.svd(cm, compute_uv=False)
        assert np.abs(s - want).max() < 1e-13


def test_generator_rejects_impossible_shapes():
    with pytest.raises(ValueError):
        workloads.bond_tensors(0, 1, 2, 7, 3)


def test_identity_update_returns_the_profile():
    l, m, r = 6, 15, 8
    center, right = workloads.bond_tensors(2, 1, l, m, r, decay=5.0)
    psi = mps.MPS([to_oracle(center[0]), to_oracle(right[0])], 0)
    before = two_site(psi)
    S = mps.apply_update(psi, 0, np.eye(9), True, True, m, 0.0)
    want = np.exp(-np.arange(m) / 5.0)
    want /= np.linalg.norm(want)
    assert len(S) == m
    assert np.abs(S - want).max() < 1e-13
    assert abs(psi.logw) < 1e-14
    assert np.abs(two_site(psi) - before).max() < 1e-13


@pytest.mark.parametrize("right_first", [True, False])
def test_gate_then_inverse_gate_restores_state(right_first):
    l, m, r = 5, 12, 6
    J, x = 0.7, 0.3
    center, right = workloads.bond_tensors(4, 1, l, m, r)
    psi = mps.MPS([to_oracle(center[0]), to_oracle(right[0])], 0)
    before = two_site(psi)
    keep = 3 * min(l, r)                   # no truncation
    mps.apply_update(psi, 0, model.gate(J, x), True, right_first, keep, 0.0)
    assert psi.logw != 0.0
    mps.apply_update(psi, 0, model.gate(J, -x), True, not right_first, keep,
                     0.0)
    assert abs(psi.logw) < 1e-13
    assert np.abs(two_site(psi) - before).max() < 1e-13


def test_pair_spin_sectors_follow_the_gate():
    # theta decomposes over the total spin S of the two physical indices;
    # the gate multiplies the S sector by exp(-x J lambda_S), lambda =
    # -2, -1, +1, so ||G theta||^2 = sum_S w_S exp(-2 x J lambda_S) with
    # w_S the sector weights of theta (unit total)
    l, m, r = 6, 14, 7
    J, x = 1.0, 0.2
    center, right = workloads.bond_tensors(6, 1, l, m, r)
    psi = mps.MPS([to_oracle(center[0]), to_oracle(right[0])], 0)
    th = two_site(psi).transpose(1, 2, 0, 3).reshape(9, -1)
    h = model.two_site_heisenberg()
    evals, evecs = np.linalg.eigh(h)
    weights = {}
    for lam in (-2.0, -1.0, 1.0):
        P = evecs[:, np.isclose(evals, lam)]
        weights[lam] = float(np.sum((P.T @ th) ** 2))
    assert abs(sum(weights.values()) - 1.0) < 1e-13
    predicted = math.log(sum(w * math.exp(-2 * x * J * lam)
                             for lam, w in weights.items()))
    mps.apply_update(psi, 0, model.gate(J, x), True, True, 3 * min(l, r), 0.0)
    assert abs(psi.logw - predicted) < 1e-12
