"""Matrix product state machinery of the hybrid method, written plainly in
FP64 NumPy (LAPACK SVD and QR).

Test infrastructure only (see the package header).

Tensor convention: site tensor T[l, s, r] (left bond, physical/ancilla
index in the S^z basis m=+1,0,-1, right bond).  One site is the
orthogonality centre; sites left of it are left-orthonormal and sites right
of it right-orthonormal.

* ``init_state``   step 1 of the Markov chain (Hybrid METTS-Ancilla
  subsection): environment product state times cluster Bell pairs
  |B_j> = d^{-1/2} sum_s |s>_P |s>_A.
* ``apply_update`` one Trotter gate (or swap) on two neighbouring sites: the
  gate breaks the MPS form, a truncated SVD restores it, discarding Schmidt
  weights up to a relative discarded weight (Results section, third source
  of error).  The state is rescaled to unit norm after every gate and the
  logarithm of the squared norm is accumulated: the sampling weight P_i
  arises from this norm bookkeeping (Hybrid METTS-Ancilla subsection).
* ``evolve``       (e^{-tau H})^M on the physical sites (step 2).
* ``measure``      <psi| S_i.S_j |psi> for every bond (step 3).
* ``collapse``     projective measurement of each environment site in turn,
  cluster sites traced (step 4).

Readings of points the paper leaves open (centre movement by QR, absorb
direction, tie rule of the truncation) are stated at each function.

Parity: evolve + measure are pinned through the exhaustive hybrid sum
(equal to the dense Trotter average, every cluster size, both bases), the
single-bond closed form, the ancilla limit and the invariants (norm,
right-orthonormality, <Q> = M_E, SU(2)); the untruncated evolution also
state by state against the update list applied to the full vector;
apply_update on a single bond through the Schmidt profile of its input,
gate inversion and the spin-sector closed form of ||G theta||^2; collapse
through detailed balance by brute force, the beta = 0 transition table and
a chi^2 test of sampled frequencies; truncation_rank through hand-made
spectra.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import model, philox

TIE_TOL = 1e-8          # relative gap below which singular values tie
NEAR_U = 1e-12          # a collapse draw this close to a threshold is flagged


@dataclass
class Stats:
    updates: int = 0
    gates: int = 0
    discarded: float = 0.0          # summed relative discarded weight
    max_chi: int = 0
    min_margin: float = math.inf    # closest relative approach of the tail
    ties: int = 0                   # truncations moved by the tie rule
    chi_hist: dict = field(default_factory=dict)
    spectra: list = None            # per-update kept spectra (if recording)


@dataclass
class MPS:
    tensors: list
    center: int
    logw: float = 0.0


# --------------------------------------------------------------------------
# step 1: initial state
# --------------------------------------------------------------------------
def init_state(lay: model.Layout, env_outcomes: dict, basis: int) -> MPS:
    """Environment sites in the product state given by env_outcomes
    (position -> outcome index in ``basis``), every cluster physical site
    in a Bell pair with the ancilla that follows it."""
    vecs = model.basis_vectors(basis)
    T = []
    p = 0
    while p < lay.length:
        if lay.is_cluster[p]:
            phys = np.zeros((1, 3, 3))
            anc = np.zeros((3, 3, 1))
            for s in range(3):
                phys[0, s, s] = 1.0 / math.sqrt(3.0)
                anc[s, s, 0] = 1.0
            T += [phys, anc]
            p += 2
        else:
            t = np.zeros((1, 3, 1))
            t[0, :, 0] = vecs[env_outcomes[p]]
            T.append(t)
            p += 1
    return MPS(T, 0, 0.0)


def initial_outcomes(lay: model.Layout, seed: int, chain: int,
                     sample: int = 0) -> dict:
    """Uniform random S^z index per environment site for the first sample
    of a chain (``sample`` = its index, 0 unless the chain is resumed)."""
    out = {}
    for p in lay.env_positions:
        u = philox.uniform(seed, chain, sample, p, philox.PURPOSE_INIT)
        out[p] = min(2, int(math.floor(3.0 * u)))
    return out


# --------------------------------------------------------------------------
# orthogonality centre
# --------------------------------------------------------------------------
def move_center(psi: MPS, target: int) -> None:
    """Move the centre with QR decompositions (no truncation)."""
    T = psi.tensors
    while psi.center < target:
        c = psi.center
        l, d, r = T[c].shape
        q, rr = np.linalg.qr(T[c].reshape(l * d, r))
        T[c] = q.reshape(l, d, q.shape[1])
        T[c + 1] = np.einsum("ab,bsc->asc", rr, T[c + 1])
        psi.center = c + 1
    while psi.center > target:
        c = psi.center
        l, d, r = T[c].shape
        q, rr = np.linalg.qr(T[c].reshape(l, d * r).T)
        T[c] = q.T.reshape(q.shape[1], d, r)
        T[c - 1] = np.einsum("asb,bc->asc", T[c - 1], rr.T)
        psi.center = c - 1


# --------------------------------------------------------------------------
# truncation
# --------------------------------------------------------------------------
def truncation_rank(s: np.ndarray, chi_max: int, cutoff: float,
                    stats: Stats | None = None) -> int:
    """Number of singular values kept.

    k_eps is the smallest k >= 1 whose discarded tail sum_{j>=k} s_j^2 is at
    most cutoff * sum_j s_j^2: the truncation error is the summed squares of
    the discarded singular values over the sum of all squares, held at a
    fixed target (Results section, third source of error).  The bond
    dimension cap gives k = min(k_eps, chi_max).

    Ties (reading of a point the paper leaves open): a run of singular
    values whose consecutive relative gaps are <= TIE_TOL has no unique
    split, so a cut never falls inside one.
      * The target sets the cut (k_eps <= chi_max): the whole run is kept,
        so the discarded weight stays within the target; if keeping it
        would pass chi_max, the cap binds and the next rule applies.
      * The cap binds: the whole run is dropped, unless it starts at the
        largest singular value (then the cut stays where the cap put it).
    """
    r = len(s)
    w = s * s
    total = float(w.sum())
    tail = np.zeros(r + 1)
    acc = 0.0
    for j in range(r - 1, -1, -1):
        acc += w[j]
        tail[j] = acc
    thr = cutoff * total
    k_eps = r
    for k in range(1, r + 1):
        if tail[k] <= thr:
            k_eps = k
            break
    k = min(k_eps, chi_max)
    if stats is not None and k == k_eps and thr > 0.0 and k_eps < r:
        m1 = abs(tail[k_eps] - thr) / thr
        m2 = abs(tail[k_eps - 1] - thr) / thr
        stats.min_margin = min(stats.min_margin, m1, m2)

    def tied(j):          # s[j - 1] and s[j] belong to one run
        return s[j - 1] - s[j] <= TIE_TOL * s[j - 1]

    if k < r and tied(k):
        moved = k
        end = k
        while end < r and tied(end):
            end += 1                       # the run ends at index end - 1
        if k_eps <= chi_max and end <= chi_max:
            moved = end                    # keep the whole run
        else:
            start = k - 1
            while start > 0 and tied(start):
                start -= 1                 # the run starts at index start
            if start > 0:
                moved = start              # drop the whole run
        if moved != k and stats is not None:
            stats.ties += 1
        k = moved
    return k


# --------------------------------------------------------------------------
# two-site update
# --------------------------------------------------------------------------
def apply_update(psi: MPS, k: int, op: np.ndarray, is_gate: bool,
                 right: bool, chi_max: int, cutoff: float,
                 stats: Stats | None = None) -> np.ndarray:
    """Apply the 9x9 operator ``op`` (index (s1,s2) -> 3*s1+s2) to sites
    (k, k+1), renormalise (gates: accumulate log of the squared norm),
    truncate, and leave the centre on k+1 (right) or k (left).  Returns
    the kept, renormalised singular values."""
    T = psi.tensors
    if psi.center < k:
        move_center(psi, k)
    elif psi.center > k + 1:
        move_center(psi, k + 1)
    A, B = T[k], T[k + 1]
    l, r = A.shape[0], B.shape[2]
    theta = np.einsum("asb,btc->astc", A, B)
    theta = np.einsum("uv,avc->auc", op, theta.reshape(l, 9, r))
    if is_gate:
        n2 = float(np.sum(theta * theta))
        psi.logw += math.log(n2)
        theta = theta / math.sqrt(n2)
    mat = theta.reshape(l * 3, 3 * r)
    U, S, Vt = np.linalg.svd(mat, full_matrices=False)
    kk = truncation_rank(S, chi_max, cutoff, stats)
    tot = float(np.sum(S * S))
    disc = float(np.sum(S[kk:] ** 2)) / tot if tot > 0 else 0.0
    U, S, Vt = U[:, :kk], S[:kk], Vt[:kk, :]
    S = S / math.sqrt(float(np.sum(S * S)))
    if right:
        T[k] = U.reshape(l, 3, kk)
        T[k + 1] = (S[:, None] * Vt).reshape(kk, 3, r)
        psi.center = k + 1
    else:
        T[k] = (U * S[None, :]).reshape(l, 3, kk)
        T[k + 1] = Vt.reshape(kk, 3, r)
        psi.center = k
    if stats is not None:
        stats.updates += 1
        stats.gates += int(is_gate)
        stats.discarded += disc
        stats.max_chi = max(stats.max_chi, kk)
        stats.chi_hist[kk] = stats.chi_hist.get(kk, 0) + 1
        if stats.spectra is not None:
            stats.spectra.append(S.copy())
    return S


def evolve(psi: MPS, sch: model.Schedule, M: int, tau: float, chi_max: int,
           cutoff: float, stats: Stats | None = None) -> None:
    """M second-order Trotter steps of exp(-tau H) on the physical sites,
    then the centre is brought back to site 0 (step 2)."""
    gates = [model.gate(J, tau / 2.0) for J in sch.couplings]
    swap = model.swap_gate()
    for u in model.evolve_updates(sch, M):
        if u.op == model.OP_SWAP:
            apply_update(psi, u.k, swap, False, u.right, chi_max, cutoff,
                         stats)
        else:
            apply_update(psi, u.k, gates[u.op], True, u.right, chi_max,
                         cutoff, stats)
    move_center(psi, 0)


# --------------------------------------------------------------------------
# step 3: measurement
# --------------------------------------------------------------------------
def _transfer(E: np.ndarray, A: np.ndarray, op=None) -> np.ndarray:
    """E'[c,d] = sum_{a,b,s,t} E[a,b] A[a,s,c] op[s,t] A[b,t,d] (bra index
    first); op=None is the identity."""
    X = np.tensordot(E, A, axes=([1], [0]))          # [a, t, d]
    if op is not None:
        X = np.tensordot(op, X, axes=([1], [1]))     # [s, a, d]
        X = X.transpose(1, 0, 2)                     # [a, s, d]
    return np.tensordot(A, X, axes=([0, 1], [0, 1]))  # [c, d]


def _environments(T: list):
    """Left environments L[p] (sites < p) and right environments R[p]
    (sites > p) of <psi|psi>, contracted explicitly (no gauge assumed)."""
    n = len(T)
    L = [np.ones((1, 1))]
    for p in range(n):
        L.append(_transfer(L[p], T[p]))
    R = [None] * n
    R[n - 1] = np.ones((1, 1))
    for p in range(n - 1, 0, -1):
        X = np.tensordot(T[p], R[p], axes=([2], [0]))          # [a, s, d]
        R[p - 1] = np.tensordot(X, T[p], axes=([1, 2], [1, 2]))  # [a, b]
    return L, R


def measure(psi: MPS, lat: model.Lattice, lay: model.Layout) -> dict:
    """Monte Carlo estimators of step 3: <S_i.S_j> for every bond of the
    lattice (in lattice bond order), the energy sum_b J_b <S_i.S_j>, the
    norm, and <Q> with Q = sum of S^z over physical sites minus sum over
    ancillas (conserved by the evolution)."""
    T = psi.tensors
    L, R = _environments(T)
    norm = float(L[len(T)][0, 0])
    terms = ((model.SZ, model.SZ, 1.0), (model.SP, model.SM, 0.5),
             (model.SM, model.SP, 0.5))
    ss = []
    for (i, j, J) in lat.bonds:
        p, q = sorted((lay.pos_of_phys[i], lay.pos_of_phys[j]))
        val = 0.0
        for (oi, oj, c) in terms:
            E = _transfer(L[p], T[p], oi)
            for m in range(p + 1, q):
                E = _transfer(E, T[m])
            E = _transfer(E, T[q], oj)
            val += c * float(np.sum(E * R[q]))
        ss.append(val / norm)
    energy = 0.0
    for b, (_, _, J) in enumerate(lat.bonds):
        energy += J * ss[b]
    qn = 0.0
    for p in range(len(T)):
        E = _transfer(L[p], T[p], model.SZ)
        v = float(np.sum(E * R[p])) / norm
        qn += -v if lay.is_ancilla[p] else v
    return {"bond_ss": ss, "energy": energy, "norm": norm, "qn": qn,
            "logw": psi.logw}


# --------------------------------------------------------------------------
# step 4: collapse
# --------------------------------------------------------------------------
def collapse(psi: MPS, lay: model.Layout, basis: int, seed: int, chain: int,
             sample: int, flags: dict | None = None) -> dict:
    """Projective measurement of every environment site in turn, in MPS
    order, in the product basis ``basis``; cluster sites (physical and
    ancilla) are traced out.  Outcome s of a site is chosen by the inverse
    CDF of its conditional probabilities with one Philox uniform number
    (strict '<').  Returns position -> outcome."""
    T = psi.tensors
    n = len(T)
    _, R = _environments(T)
    vecs = model.basis_vectors(basis)
    out = {}
    Mt = T[0]
    for k in range(n):
        if lay.is_cluster[k]:
            l, d, r = Mt.shape
            _, rr = np.linalg.qr(Mt.reshape(l * d, r))
            if k + 1 < n:
                Mt = np.einsum("ab,bsc->asc", rr, T[k + 1])
            continue
        amp = np.einsum("ts,asb->atb", vecs, Mt)
        p = np.array([float(np.sum((amp[:, t, :] @ R[k]) * amp[:, t, :]))
                      for t in range(3)])
        p = np.maximum(p, 0.0)
        cum = np.cumsum(p) / p.sum()
        cum[-1] = 1.0
        u = philox.uniform(seed, chain, sample, k, philox.PURPOSE_COLLAPSE)
        s = int(np.argmax(u < cum))
        if flags is not None and float(np.min(np.abs(u - cum))) < NEAR_U:
            flags["near"] = flags.get("near", 0) + 1
        out[k] = s
        v = amp[:, s, :] / math.sqrt(p[s])
        if k + 1 < n:
            Mt = np.einsum("ab,bsc->asc", v, T[k + 1])
    return out


def outcome_probability(psi: MPS, lay: model.Layout, basis: int,
                        outcomes: dict) -> float:
    """<psi| Pi_j |psi> / <psi|psi> for the environment product state j
    given by ``outcomes`` (position -> outcome) in ``basis``, with
    Pi_j = |j><j|_E (x) 1_C (Discussion of Detailed Balance).  Computed by
    contracting the projected state with itself, no sampling."""
    T = psi.tensors
    vecs = model.basis_vectors(basis)
    E = np.ones((1, 1))
    N = np.ones((1, 1))
    for k in range(len(T)):
        N = _transfer(N, T[k])
        if lay.is_cluster[k]:
            E = _transfer(E, T[k])
        else:
            v = vecs[outcomes[k]]
            E = _transfer(E, T[k], np.outer(v, v))
    return float(E[0, 0] / N[0, 0])
