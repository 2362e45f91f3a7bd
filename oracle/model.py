"""Model definitions for the oracle: spin-1 operators, the S=1 two-leg ladder,
the two-site imaginary-time gate, the hybrid MPS site layout and the
second-order Trotter update list.

Test infrastructure only (see the package header).  Every quantity here is
written from its definition in Chen & Stoudenmire, arXiv:1910.09142:

* Hamiltonian: Results section, ladder Hamiltonian (legs J, rungs J_perp,
  open boundaries), spin S=1 so d=3 (Ancilla Method subsection).
* Trotter: Ancilla Method subsection, e^{-H beta/2} = (e^{-H tau})^M with
  tau = beta/(2M); second-order Trotter-Suzuki with tau=0.05 (Results
  section, sources of error).
* Layout: physical/ancilla interleaving (Ancilla Method subsection), a
  contiguous central cluster paired with ancillas (Hybrid METTS-Ancilla
  subsection and Fig. "initial").

Parity: the gate is pinned to scipy.linalg.expm and to SU(2) invariance; the
Trotter update list is pinned through the dense Trotter product (exact.py)
and exhaustive hybrid sums in tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

D = 3  # physical dimension of a spin-1 site

# --------------------------------------------------------------------------
# spin-1 operators in the S^z eigenbasis ordered m = +1, 0, -1
# --------------------------------------------------------------------------
SZ = np.diag([1.0, 0.0, -1.0])
SP = np.array([[0.0, math.sqrt(2.0), 0.0],
               [0.0, 0.0, math.sqrt(2.0)],
               [0.0, 0.0, 0.0]])
SM = SP.T.copy()
SX = 0.5 * (SP + SM)
ID3 = np.eye(3)

# Eigenvectors of S^x written in the S^z basis, ordered by eigenvalue
# +1, 0, -1, first component positive.  Row s is the vector for outcome s.
SX_BASIS = np.array([[0.5, 1.0 / math.sqrt(2.0), 0.5],
                     [1.0 / math.sqrt(2.0), 0.0, -1.0 / math.sqrt(2.0)],
                     [0.5, -1.0 / math.sqrt(2.0), 0.5]])
SZ_BASIS = np.eye(3)


def basis_vectors(basis: int) -> np.ndarray:
    """Rows are the product-state vectors of outcome 0,1,2 (eigenvalue
    +1,0,-1) of S^z (basis 0) or S^x (basis 1)."""
    if basis == 0:
        return SZ_BASIS
    if basis == 1:
        return SX_BASIS
    raise ValueError("basis must be 0 (S^z) or 1 (S^x)")


def two_site_heisenberg() -> np.ndarray:
    """h = S_1 . S_2 on C^3 (x) C^3, index (s1, s2) -> 3*s1 + s2."""
    return (np.kron(SZ, SZ) + 0.5 * (np.kron(SP, SM) + np.kron(SM, SP)))


def gate(J: float, x: float) -> np.ndarray:
    """exp(-x J S_1.S_2) as a 9x9 matrix.

    S_1.S_2 has eigenvalues -2, -1, +1 on total spin 0, 1, 2 (multiplicity
    1, 3, 5), so the exponential is a sum of the three spectral projectors
    P_S weighted by exp(-x J lambda_S).  The projectors are the Lagrange
    polynomials of h in its three eigenvalues.
    """
    h = two_site_heisenberg()
    one = np.eye(9)
    p0 = (h @ h - one) / 3.0                 # lambda = -2
    p1 = -(h + 2.0 * one) @ (h - one) / 2.0  # lambda = -1
    p2 = (h + 2.0 * one) @ (h + one) / 6.0   # lambda = +1
    return (math.exp(2.0 * x * J) * p0 + math.exp(x * J) * p1
            + math.exp(-x * J) * p2)


def swap_gate() -> np.ndarray:
    """The 9x9 permutation exchanging the two sites."""
    s = np.zeros((9, 9))
    for a in range(3):
        for b in range(3):
            s[3 * b + a, 3 * a + b] = 1.0
    return s


# --------------------------------------------------------------------------
# lattice
# --------------------------------------------------------------------------
@dataclass
class Lattice:
    """A spin-1 Hamiltonian H = sum_b J_b S_i.S_j on n_phys sites together
    with the order of the physical sites along the MPS and the cluster
    mask (physical sites purified by an ancilla partner)."""
    n_phys: int
    bonds: list            # list of (i, j, J) with physical ids i != j
    order: list            # physical ids in MPS order
    in_cluster: list       # bool per physical id
    name: str = ""


def ladder(L: int, J_leg: float = 1.0, J_rung: float = 1.0, W: int = 0,
           ordering: str = "snake") -> Lattice:
    """S=1 two-leg ladder with open boundaries (Results section).

    Physical site (column c, leg l) has id 2c+l.  Bonds: the rung
    (c,0)-(c,1) with J_rung for every column, the legs (c,l)-(c+1,l) with
    J_leg.  Bond list order: all rungs by column, then leg 0, then leg 1.
    The cluster is W contiguous central columns c0..c0+W-1 with
    c0 = (L-W)//2 (Hybrid METTS-Ancilla subsection: contiguous cluster at
    the spatial centre).  MPS order "snake": column c lists leg 0 then leg 1
    when c is even, leg 1 then leg 0 when c is odd; "zigzag": always leg 0
    then leg 1.
    """
    bonds = []
    for c in range(L):
        bonds.append((2 * c, 2 * c + 1, float(J_rung)))
    for leg in range(2):
        for c in range(L - 1):
            bonds.append((2 * c + leg, 2 * (c + 1) + leg, float(J_leg)))
    order = []
    for c in range(L):
        if ordering == "snake" and c % 2 == 1:
            order += [2 * c + 1, 2 * c]
        elif ordering in ("snake", "zigzag"):
            order += [2 * c, 2 * c + 1]
        else:
            raise ValueError(ordering)
    c0 = (L - W) // 2
    in_cluster = [False] * (2 * L)
    for c in range(c0, c0 + W):
        in_cluster[2 * c] = True
        in_cluster[2 * c + 1] = True
    return Lattice(2 * L, bonds, order, in_cluster,
                   name=f"ladder{L}x2_W{W}_{ordering}")


def chain(N: int, J: float = 1.0, cluster=None) -> Lattice:
    """Open S=1 chain (used for small checks)."""
    bonds = [(i, i + 1, float(J)) for i in range(N - 1)]
    inc = [False] * N
    for i in (cluster or []):
        inc[i] = True
    return Lattice(N, bonds, list(range(N)), inc, name=f"chain{N}")


# --------------------------------------------------------------------------
# hybrid MPS layout
# --------------------------------------------------------------------------
@dataclass
class Layout:
    """MPS sites: physical sites in lattice.order, each cluster site followed
    immediately by its ancilla partner."""
    length: int
    phys_of_pos: list   # physical id, or -1 for an ancilla
    pos_of_phys: list   # MPS position of each physical id
    is_ancilla: list
    is_cluster: list    # physical cluster site or ancilla
    env_positions: list  # MPS positions of environment sites, ascending


def layout(lat: Lattice) -> Layout:
    phys_of_pos, is_anc, is_cl = [], [], []
    pos_of_phys = [-1] * lat.n_phys
    for i in lat.order:
        pos_of_phys[i] = len(phys_of_pos)
        phys_of_pos.append(i)
        is_anc.append(False)
        is_cl.append(bool(lat.in_cluster[i]))
        if lat.in_cluster[i]:
            phys_of_pos.append(-1)
            is_anc.append(True)
            is_cl.append(True)
    env = [p for p in range(len(phys_of_pos)) if not is_cl[p]]
    return Layout(len(phys_of_pos), phys_of_pos, pos_of_phys, is_anc, is_cl,
                  env)


# --------------------------------------------------------------------------
# Trotter update list
# --------------------------------------------------------------------------
OP_SWAP = -1


@dataclass
class Update:
    k: int          # acts on MPS sites (k, k+1)
    op: int         # index into the distinct couplings, or OP_SWAP
    right: bool     # absorb the singular values to the right (centre -> k+1)


@dataclass
class Schedule:
    couplings: list            # distinct J values, in first-appearance order
    mps_bonds: list            # (p, q, J index) sorted by (p, q)
    half: list                 # updates of the forward half-sweep
    step: list = field(default_factory=list)  # forward + reversed


def schedule(lat: Lattice, lay: Layout | None = None) -> Schedule:
    """Second-order Trotter step as a list of nearest-neighbour updates.

    A bond (i,j) at MPS positions p<q is applied by swapping the content of
    site p rightwards to q-1, applying the gate on (q-1,q), and swapping it
    back.  The forward half-sweep takes the bonds sorted by (p,q); one step
    is the forward half-sweep followed by the same updates in reverse
    order, so the step operator is palindromic (second order) and each
    bond's gate uses half the time step.
    """
    lay = lay or layout(lat)
    couplings = []
    mb = []
    for (i, j, J) in lat.bonds:
        if J not in couplings:
            couplings.append(J)
        p, q = sorted((lay.pos_of_phys[i], lay.pos_of_phys[j]))
        mb.append((p, q, couplings.index(J)))
    mb.sort(key=lambda t: (t[0], t[1]))
    ops = []
    for (p, q, jx) in mb:
        for k in range(p, q - 1):
            ops.append((k, OP_SWAP))
        ops.append((q - 1, jx))
        for k in range(q - 2, p - 1, -1):
            ops.append((k, OP_SWAP))
    step_ops = ops + ops[::-1]
    return Schedule(couplings, mb, ops, step_ops)


def absorb_right(k: int, k_next: int) -> bool:
    """Direction rule: move the orthogonality centre towards the next
    update, to the right when the next update starts at or right of k."""
    return k_next >= k


def evolve_updates(sch: Schedule, M: int) -> list:
    """The full list of updates for M Trotter steps with absorb directions.
    The update after the last one is taken at k=0 (the centre is finally
    brought to site 0)."""
    seq = sch.step * M
    out = []
    for t, (k, op) in enumerate(seq):
        kn = seq[t + 1][0] if t + 1 < len(seq) else 0
        out.append(Update(k, op, absorb_right(k, kn)))
    return out


def trotter_steps(beta: float, tau: float) -> int:
    """M = beta/(2 tau) must be an integer (Ancilla Method subsection)."""
    m = beta / (2.0 * tau)
    M = int(round(m))
    if M < 0 or abs(m - M) > 1e-9 * max(1.0, abs(m)):
        raise ValueError("beta/(2 tau) must be an integer")
    return M
