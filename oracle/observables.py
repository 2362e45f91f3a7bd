"""Long-range observables of one sample (Results section, susceptibility):
correlators <S_i.S_j> of arbitrary spin pairs and the susceptibility
estimator built from them.

Test infrastructure: the reference the GPU path is checked against, never
called by it.

Parity: pinned against dense exact diagonalisation of sum_{j in C} sum_i
S_j.S_i through the exhaustive hybrid identity (any centre set C, both
bases) and against product states, where <S_i.S_j> = m_i m_j.
"""
from __future__ import annotations

from . import model, mps


def pair_correlations(psi: mps.MPS, lat: model.Lattice, lay: model.Layout,
                      pairs) -> list:
    """<S_i.S_j> for physical-site pairs (i, j) of the sample; i == j gives
    s(s+1) = 2.  The strings are those of the bond measurement: a lattice
    whose bonds are the requested pairs."""
    distinct = sorted({(i, j) for (i, j) in pairs if i != j})
    vals = {}
    if distinct:
        pseudo = model.Lattice(lat.n_phys, [(i, j, 1.0) for (i, j) in distinct],
                               lat.order, lat.in_cluster)
        r = mps.measure(psi, pseudo, lay)
        vals = dict(zip(distinct, r["bond_ss"]))
    return [2.0 if i == j else vals[(i, j)] for (i, j) in pairs]


def susceptibility(psi: mps.MPS, lat: model.Lattice, lay: model.Layout,
                   beta: float, center) -> float:
    """chi = (beta/3) (1/|C|) sum_{j in C} sum_{i in all} <S_j.S_i>, i
    running over every physical site including j (Results section: the
    paper takes C = the middle 6 x 2 sites of the ladder)."""
    center = list(center)
    pairs = [(j, i) for j in center for i in range(lat.n_phys)]
    return beta / 3.0 * sum(pair_correlations(psi, lat, lay, pairs)) / len(center)
