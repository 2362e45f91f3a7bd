"""Long-range observables of one sample (Results section, susceptibility):
correlators <S_i.S_j> of arbitrary spin pairs and the susceptibility
estimator built from them; and the sample moments of the per-bond
estimators over many samples (the variance study of Section Entanglement
and Cost of Hybrid States).

Test infrastructure: the reference the GPU path is checked against, never
called by it.

Parity: pinned against dense exact diagonalisation of sum_{j in C} sum_i
S_j.S_i through the exhaustive hybrid identity (any centre set C, both
bases) and against product states, where <S_i.S_j> = m_i m_j.
sample_moments is the textbook definition, pinned by closed forms (a
two-valued sample, a constant one, a hand-computed one).
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


def sample_moments(values):
    """Mean and unbiased sample variance of each column of `values` (rows:
    samples, e.g. every chain's every measurement; columns: bonds):
    mean_b = sum_s x_sb / n, var_b = sum_s (x_sb - mean_b)^2 / (n - 1).
    The Markov chain draws product states with probability P_i / sum_j
    P_j, so the samples are weighted equally."""
    rows = [list(map(float, r)) for r in values]
    n = len(rows)
    if n < 2:
        raise ValueError("the sample variance needs at least two samples")
    cols = len(rows[0])
    mean = [sum(r[b] for r in rows) / n for b in range(cols)]
    var = [sum((r[b] - mean[b]) ** 2 for r in rows) / (n - 1)
           for b in range(cols)]
    return n, mean, var
