"""Exact reference quantities on small lattices: the thermal average by exact
diagonalisation and the dense (state-vector) Trotter product.

Test infrastructure only (see the package header).

* ``thermal_energy`` follows the canonical-ensemble definition
  <A> = Tr[A e^{-beta H}]/Z (Hybrid Purification-Sampling Method section,
  density-matrix and thermal-average equations).
* ``trotter_operator`` builds (e^{-tau H})^M in its second-order
  palindromic form from the same bond order as the MPS update list, but as
  a dense 3^N x 3^N matrix on physical sites only (no ancillas, no swaps,
  no MPS).  ``trotter_average`` = Tr[A U^2]/Tr[U^2], the symmetric form of
  the thermal average with U = e^{-beta H/2} replaced by its Trotter
  product.

Pins: the ED energies are checked against the closed form of a single bond,
the high-temperature series and a second diagonalisation of the 2x3 ladder
written independently, sector by sector in total S^z; the Trotter product
against tau^2 convergence to ED.
"""
from __future__ import annotations

import numpy as np

from . import model


def _site_op(op: np.ndarray, i: int, n: int) -> np.ndarray:
    out = np.ones((1, 1))
    for s in range(n):
        out = np.kron(out, op if s == i else np.eye(3))
    return out


def bond_operator(i: int, j: int, n: int) -> np.ndarray:
    """S_i . S_j on n spin-1 sites (dense)."""
    return (_site_op(model.SZ, i, n) @ _site_op(model.SZ, j, n)
            + 0.5 * (_site_op(model.SP, i, n) @ _site_op(model.SM, j, n)
                     + _site_op(model.SM, i, n) @ _site_op(model.SP, j, n)))


def hamiltonian(lat: model.Lattice) -> np.ndarray:
    n = lat.n_phys
    H = np.zeros((3 ** n, 3 ** n))
    for (i, j, J) in lat.bonds:
        H += J * bond_operator(i, j, n)
    return H


def thermal_average(lat: model.Lattice, beta: float, ops: list) -> list:
    """<A> = Tr[A e^{-beta H}]/Tr[e^{-beta H}] for each A in ops (exact
    diagonalisation; energies shifted by the ground energy for stability)."""
    H = hamiltonian(lat)
    w, v = np.linalg.eigh(H)
    p = np.exp(-beta * (w - w[0]))
    Z = p.sum()
    out = []
    for A in ops:
        diag = np.einsum("ij,ik,kj->j", v, A, v)
        out.append(float((p * diag).sum() / Z))
    return out


def thermal_energy(lat: model.Lattice, beta: float) -> float:
    H = hamiltonian(lat)
    w = np.linalg.eigvalsh(H)
    p = np.exp(-beta * (w - w[0]))
    return float((p * w).sum() / p.sum())


def ground_energy(lat: model.Lattice) -> float:
    return float(np.linalg.eigvalsh(hamiltonian(lat))[0])


def _embed_two_site(g9: np.ndarray, i: int, j: int, n: int) -> np.ndarray:
    """Dense operator acting as the 9x9 matrix g9 on sites (i, j)."""
    dim = 3 ** n
    out = np.zeros((dim, dim))
    g = g9.reshape(3, 3, 3, 3)
    for col in range(dim):
        digits = [(col // 3 ** (n - 1 - s)) % 3 for s in range(n)]
        a, b = digits[i], digits[j]
        for c in range(3):
            for d in range(3):
                val = g[c, d, a, b]
                if val == 0.0:
                    continue
                dd = list(digits)
                dd[i], dd[j] = c, d
                row = 0
                for s in range(n):
                    row = row * 3 + dd[s]
                out[row, col] += val
    return out


def trotter_operator(lat: model.Lattice, tau: float, M: int) -> np.ndarray:
    """(U_step)^M with U_step the palindromic product of bond gates
    exp(-(tau/2) J h_b): bonds in the MPS update-list order (sorted by
    their MPS positions), then the same bonds in reverse order."""
    n = lat.n_phys
    sch = model.schedule(lat)
    lay = model.layout(lat)
    phys = lay.phys_of_pos
    mats = []
    for (p, q, jx) in sch.mps_bonds:
        J = sch.couplings[jx]
        mats.append(_embed_two_site(model.gate(J, tau / 2.0), phys[p],
                                    phys[q], n))
    step = np.eye(3 ** n)
    for m in mats:                 # forward half-sweep applied first
        step = m @ step
    for m in reversed(mats):       # then the reversed half-sweep
        step = m @ step
    return np.linalg.matrix_power(step, M)


def trotter_average(lat: model.Lattice, beta: float, tau: float,
                    ops: list) -> list:
    """Tr[A U^2]/Tr[U^2] with U the Trotter product for beta/2."""
    M = model.trotter_steps(beta, tau)
    U = trotter_operator(lat, tau, M)
    U2 = U @ U
    z = np.trace(U2)
    return [float(np.trace(A @ U2) / z) for A in ops]


def trotter_energy(lat: model.Lattice, beta: float, tau: float) -> float:
    return trotter_average(lat, beta, tau, [hamiltonian(lat)])[0]


def single_bond_energy(J: float, beta: float) -> float:
    """Closed form for a single bond J S_1.S_2: its levels are -2J (total
    spin 0, 1 state), -J (spin 1, 3 states) and +J (spin 2, 5 states)."""
    e = np.array([-2.0 * J, -J, J])
    g = np.array([1.0, 3.0, 5.0])
    w = g * np.exp(-beta * (e - e.min()))
    return float((w * e).sum() / w.sum())


def high_t_energy(lat: model.Lattice, beta: float) -> float:
    """Leading high-temperature series of the energy for a lattice without
    triangles: -sum_b [(4/3) J_b^2 beta + (1/3) J_b^3 beta^2] + O(beta^3).
    (<(S.S)^2>_0 = 4/3 and <(S.S)^3>_0 = -2/3 for two spin-1 sites.)"""
    s = 0.0
    for (_, _, J) in lat.bonds:
        s += (4.0 / 3.0) * J * J * beta + (1.0 / 3.0) * J ** 3 * beta ** 2
    return -s
