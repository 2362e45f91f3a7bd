"""Seeded synthetic inputs: the S=1 two-leg ladder workloads and their run
parameters.  Holds no arithmetic of the method (the lattice is the input
Hamiltonian of the C ABI; random product states are drawn inside the
library by Philox).  Shared by tests, smoke() and bench.py.

Ladder (Results section): sites (column c, leg l) with id 2c+l, rungs
(c,0)-(c,1) with J_rung, legs (c,l)-(c+1,l) with J_leg, open boundaries.
Bond order: rungs by column, then leg 0, then leg 1.  MPS order "snake":
column c lists leg 0 then leg 1 for even c, leg 1 then leg 0 for odd c.
Cluster: W central columns starting at (L-W)//2.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class Workload:
    name: str
    L: int
    W: int
    J_leg: float
    J_rung: float
    beta: float
    tau: float
    chi_max: int
    cutoff: float
    n_chains: int
    n_samples: int
    seed: int = 0


# The five ladder workloads (sizes as stated for each one).
C1 = Workload("ladder2x3_W1_beta1_chi32", 3, 1, 1.0, 1.0, 1.0, 0.1, 32,
              1e-12, 1, 20)
C2 = Workload("ladder2x8_W2_beta5_chi128", 8, 2, 1.0, 1.0, 5.0, 0.05, 128,
              1e-12, 1, 100)
C3 = Workload("ladder2x16_W2_Jr0.5_beta5_chi256", 16, 2, 1.0, 0.5, 5.0,
              0.05, 256, 1e-10, 1, 2)
C4 = Workload("ladder2x16_W2_Jr0.5_beta5_chi256_batch256", 16, 2, 1.0, 0.5,
              5.0, 0.05, 256, 1e-10, 256, 1)
C5 = Workload("ladder2x32_W4_beta10_chi512_batch64", 32, 4, 1.0, 1.0, 10.0,
              0.05, 512, 1e-10, 64, 1)
ALL = {w.name: w for w in (C1, C2, C3, C4, C5)}


def ladder_arrays(L: int, J_leg: float, J_rung: float, W: int,
                  ordering: str = "snake"):
    """(n_phys, bonds [(i, j, J)], mps order, cluster mask)."""
    bonds = [(2 * c, 2 * c + 1, float(J_rung)) for c in range(L)]
    for leg in range(2):
        bonds += [(2 * c + leg, 2 * (c + 1) + leg, float(J_leg))
                  for c in range(L - 1)]
    order = []
    for c in range(L):
        if ordering == "snake" and c % 2 == 1:
            order += [2 * c + 1, 2 * c]
        else:
            order += [2 * c, 2 * c + 1]
    c0 = (L - W) // 2
    mask = [0] * (2 * L)
    for c in range(c0, c0 + W):
        mask[2 * c] = mask[2 * c + 1] = 1
    return 2 * L, bonds, order, mask


def central_sites(L: int, ncols: int = 6):
    """Physical ids of the middle ncols x 2 sites of a 2 x L ladder (the
    centre set of the susceptibility estimator; the paper uses 6 x 2)."""
    c0 = (L - ncols) // 2
    return [2 * c + leg for c in range(c0, c0 + ncols) for leg in range(2)]


def mps_length(L: int, W: int) -> int:
    return 2 * L + 2 * W


# Single-gate workload: every update at chi_l = chi_m = chi_r = 256, the
# gate exp(-(tau/2) J S.S) with J = 1, tau = 0.05, chi_max 256, cutoff
# 1e-10 (the chi = 256 ladder's half-step gate and truncation).
@dataclass(frozen=True)
class BondWorkload:
    name: str
    chi: int
    J: float
    x: float
    chi_max: int
    cutoff: float
    decay: float
    seed: int = 0


M1 = BondWorkload("bond_chi256_gate_J1_x0.025", 256, 1.0, 0.025, 256, 1e-10,
                  24.0)


def _haar_columns(rng, rows: int, cols: int):
    """rows x cols matrix with orthonormal columns, Haar distributed (QR of
    a Gaussian matrix, signs fixed by the diagonal of R)."""
    import numpy as np
    q, r = np.linalg.qr(rng.standard_normal((rows, cols)))
    return q * np.sign(np.diag(r))[None, :]


def bond_tensors(seed: int, n_chains: int, chi_l: int, chi_m: int,
                 chi_r: int, decay: float = 24.0):
    """Synthetic bond of an MPS for each chain, in the layout T[s, a, b] of
    the C ABI: the centre C (3, chi_l, chi_m) with Schmidt values
    sigma_j proportional to exp(-j / decay) on its right bond (C = Q1
    diag(sigma) Q2 as a (chi_l*3) x chi_m matrix, Q1 and Q2 Haar), and a
    right-orthonormal B (3, chi_m, chi_r) (rows of a Haar isometry).
    Needs 3 chi_l >= chi_m and 3 chi_r >= chi_m.  numpy Generator on
    Philox(seed)."""
    import numpy as np
    if 3 * chi_l < chi_m or 3 * chi_r < chi_m:
        raise ValueError("3 chi_l >= chi_m and 3 chi_r >= chi_m needed")
    rng = np.random.Generator(np.random.Philox(seed))
    sigma = np.exp(-np.arange(chi_m) / decay)
    sigma /= np.sqrt(np.sum(sigma * sigma))
    center = np.empty((n_chains, 3, chi_l, chi_m))
    right = np.empty((n_chains, 3, chi_m, chi_r))
    for c in range(n_chains):
        q1 = _haar_columns(rng, 3 * chi_l, chi_m)
        q2 = _haar_columns(rng, chi_m, chi_m)
        cm = (q1 * sigma[None, :]) @ q2.T            # rows (a, s)
        center[c] = cm.reshape(chi_l, 3, chi_m).transpose(1, 0, 2)
        bm = _haar_columns(rng, 3 * chi_r, chi_m).T  # columns (s, c)
        right[c] = bm.reshape(chi_m, 3, chi_r).transpose(1, 0, 2)
    return center, right
