"""The hybrid METTS-ancilla Markov chain (Hybrid METTS-Ancilla subsection,
Markov Chain Sampling Algorithm steps 1-4), and the exhaustive sum over
environment product states that the chain samples.

Test infrastructure only (see the package header).

Readings of points the paper leaves open:

* Collapse basis: sample n collapses its environment in S^z when n is even
  and in S^x when n is odd; sample 0 starts from a uniformly random S^z
  product state (one Philox draw per environment site).  With
  ``z_only`` every collapse is in S^z: the policy that keeps each
  evolution inside one sector of the total S^z (with the ancillas counted
  with flipped sign) while the sector still changes from sample to sample
  (Exploiting Conserved Quantum Numbers subsection).
* Estimators are plain sample means over the chain (the chain visits
  product states i with probability P_i/Z, where P_i is the squared norm of
  e^{-beta H/2}|i>_E|B>_C; eq. (eq2)).

``exhaustive_average`` evaluates sum_i P_i <psi_i|A|psi_i> / sum_i P_i over
all 3^{N_E} environment product states, with P_i = exp(logw_i) from the
norm bookkeeping of the evolution.  Without truncation it equals
Tr[A U^2]/Tr[U^2] for the Trotter product U, for every cluster size and
every orthonormal product basis: a pin of the whole MPS path against the
dense Trotter product.

Parity unpinned: ``run_chain`` statistics beyond brute-force size (long
chains agree with exact results only within error bars; the mean of 20
samples on the 2x3 ladder is checked against ED within its error bar).
Single samples of a chain are pinned through the MPS functions.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import model, mps


def run_sample(lat, lay, sch, M, tau, chi_max, cutoff, env, basis,
               stats=None):
    psi = mps.init_state(lay, env, basis)
    mps.evolve(psi, sch, M, tau, chi_max, cutoff, stats)
    return psi, mps.measure(psi, lat, lay)


def run_chain(lat: model.Lattice, beta: float, tau: float, chi_max: int,
              cutoff: float, n_samples: int, seed: int, chain: int = 0,
              env0: dict | None = None, basis0: int = 0,
              record_spectra: bool = False, first_sample: int = 0,
              z_only: bool = False) -> list:
    """Samples first_sample .. first_sample + n_samples - 1 of one Markov
    chain (a chain resumes at first_sample from the product state env0 of
    the previous collapse).  Each record holds the initial product state,
    the estimators and the collapse outcomes."""
    lay = model.layout(lat)
    sch = model.schedule(lat, lay)
    M = model.trotter_steps(beta, tau)
    env = dict(env0) if env0 is not None else mps.initial_outcomes(
        lay, seed, chain, first_sample)
    basis = basis0
    out = []
    for n in range(first_sample, first_sample + n_samples):
        st = mps.Stats()
        if record_spectra:
            st.spectra = []
        psi, meas = run_sample(lat, lay, sch, M, tau, chi_max, cutoff, env,
                               basis, st)
        cb = 0 if z_only else n % 2
        flags = {}
        new_env = mps.collapse(psi, lay, cb, seed, chain, n, flags)
        out.append({"sample": n, "env": dict(env), "basis": basis,
                    "energy": meas["energy"], "bond_ss": meas["bond_ss"],
                    "logw": meas["logw"], "qn": meas["qn"],
                    "norm": meas["norm"], "outcomes": new_env,
                    "collapse_basis": cb, "near": flags.get("near", 0),
                    "stats": st})
        env, basis = new_env, cb
    return out


def exhaustive_average(lat: model.Lattice, beta: float, tau: float,
                       chi_max: int, cutoff: float, basis: int = 0) -> dict:
    """sum_i P_i <A>_i / sum_i P_i over every environment product state in
    ``basis`` for A = H and each bond S_i.S_j; weights are shifted by the
    largest log-weight before exponentiation."""
    lay = model.layout(lat)
    sch = model.schedule(lat, lay)
    M = model.trotter_steps(beta, tau)
    recs = []
    for combo in itertools.product(range(3), repeat=len(lay.env_positions)):
        env = dict(zip(lay.env_positions, combo))
        psi, meas = run_sample(lat, lay, sch, M, tau, chi_max, cutoff, env,
                               basis)
        recs.append(meas)
    lw = np.array([r["logw"] for r in recs])
    w = np.exp(lw - lw.max())
    z = w.sum()
    energy = float(sum(wi * r["energy"] for wi, r in zip(w, recs)) / z)
    nb = len(lat.bonds)
    ss = [float(sum(wi * r["bond_ss"][b] for wi, r in zip(w, recs)) / z)
          for b in range(nb)]
    return {"energy": energy, "bond_ss": ss, "logw": lw, "records": recs}


def estimate(values, n_bins: int = 0):
    """Mean and standard error (optionally from n_bins equal bins)."""
    x = np.asarray(values, dtype=float)
    if n_bins and len(x) >= n_bins:
        m = len(x) // n_bins
        x = x[: m * n_bins].reshape(n_bins, m).mean(axis=1)
    mean = float(x.mean())
    err = float(x.std(ddof=1) / math.sqrt(len(x))) if len(x) > 1 else math.inf
    return mean, err
