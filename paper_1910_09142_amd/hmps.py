"""Thin ctypes binding of libhmps.so (the C ABI declared in include/hmps.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch supplies the device workspace (one uint8 tensor) and the
stream; nothing here computes physics.  The binding fails loudly when the
library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhmps.so")

HMPS_OK = 0
HMPS_E_INVALID = 1
HMPS_E_NOMEM = 2
HMPS_E_DEVICE = 3
HMPS_E_STATE = 4
HMPS_E_NUMERIC = 5
PREC_FP64 = 0
PREC_MIXED_FP32 = 1
PREC_MIXED_BF16X3 = 2      # declared by the ABI, rejected by hmps_create
MEASURE_ENERGY = 1
MEASURE_BONDS = 2
MEASURE_LOGW = 4
MEASURE_QN = 8
MEASURE_ALL = 15
MEASURE_ACCUMULATE = 16    # add to the device-side moments (not an output)
SYM_NONE = 0
SYM_U1 = 1                 # charge-conserving (block-sparse) updates

EXPORTS = [
    "hmps_workspace_bytes", "hmps_create", "hmps_init_cluster_env",
    "hmps_evolve", "hmps_measure", "hmps_collapse_resample", "hmps_stats",
    "hmps_bond_dims", "hmps_destroy", "hmps_last_error", "hmps_gate",
    "hmps_schedule", "hmps_svd_probe", "hmps_measure_pairs",
    "hmps_susceptibility", "hmps_read_site", "hmps_load_bond",
    "hmps_apply_gate", "hmps_init_cluster_env_at", "hmps_evolve_updates",
    "hmps_last_spectrum", "hmps_svd_probe_noalloc", "hmps_moments_reset",
    "hmps_bond_moments", "hmps_workspace_bytes_sym", "hmps_bond_charges",
    "hmps_set_width_rule",
]


class hmps_options(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("max_chains", C.c_int32), ("max_sites", C.c_int32),
                ("chi_cap", C.c_int32), ("max_bonds", C.c_int32),
                ("precision", C.c_int32), ("max_sweeps", C.c_int32),
                ("jacobi_tol", C.c_double),
                ("progress", C.c_void_p), ("progress_user", C.c_void_p),
                ("symmetry", C.c_int32), ("max_blocks", C.c_int32)]


PROGRESS_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int64, C.c_int64)


class hmps_lattice(C.Structure):
    _fields_ = [("n_phys", C.c_int32), ("n_bonds", C.c_int32),
                ("bond_i", C.POINTER(C.c_int32)),
                ("bond_j", C.POINTER(C.c_int32)),
                ("bond_J", C.POINTER(C.c_double)),
                ("mps_order", C.POINTER(C.c_int32)),
                ("in_cluster", C.POINTER(C.c_uint8))]


class hmps_stats_t(C.Structure):
    _fields_ = [("updates", C.c_int64), ("gate_updates", C.c_int64),
                ("move_updates", C.c_int64), ("jacobi_sweeps", C.c_int64),
                ("max_chi", C.c_int32), ("n_chains", C.c_int32),
                ("n_sites", C.c_int32), ("n_env", C.c_int32),
                ("sample", C.c_int64), ("discarded_weight", C.c_double),
                ("evolve_seconds", C.c_double), ("algo_flops", C.c_double),
                ("svd_flops", C.c_double), ("svd_seconds", C.c_double),
                ("round_launches", C.c_int64), ("svd_bytes", C.c_double),
                ("center", C.c_int64), ("evolve_pos", C.c_int64),
                ("jacobi_sweeps_fp32", C.c_int64),
                ("wide_launches", C.c_int64), ("u1_blocks", C.c_int64),
                ("split_launches", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libhmps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with "
            "`python -m paper_1910_09142_amd.build` (no fallback exists)")
    lib = C.CDLL(path)
    P = C.POINTER
    lib.hmps_workspace_bytes.restype = C.c_size_t
    lib.hmps_workspace_bytes.argtypes = [C.c_int32] * 4
    lib.hmps_workspace_bytes_sym.restype = C.c_size_t
    lib.hmps_workspace_bytes_sym.argtypes = [C.c_int32] * 6
    lib.hmps_bond_charges.argtypes = [C.c_void_p, C.c_int32, C.c_int32,
                                      P(C.c_int32)]
    lib.hmps_set_width_rule.argtypes = [C.c_void_p, C.c_int32, P(C.c_int32),
                                        P(C.c_int32)]
    lib.hmps_create.argtypes = [P(C.c_void_p), P(hmps_options)]
    lib.hmps_init_cluster_env.argtypes = [C.c_void_p, P(hmps_lattice),
                                          C.c_int32, C.c_uint64,
                                          P(C.c_uint8), C.c_int32]
    lib.hmps_init_cluster_env_at.argtypes = [
        C.c_void_p, P(hmps_lattice), C.c_int32, C.c_uint64, C.c_uint64,
        C.c_int64, P(C.c_uint8), C.c_int32]
    lib.hmps_evolve.argtypes = [C.c_void_p, C.c_double, C.c_double,
                                C.c_int32, C.c_double]
    lib.hmps_evolve_updates.argtypes = [C.c_void_p, C.c_double, C.c_double,
                                        C.c_int32, C.c_double, C.c_int64,
                                        C.c_int64]
    lib.hmps_last_spectrum.argtypes = [C.c_void_p, C.c_int32, P(C.c_int32),
                                       P(C.c_double)]
    lib.hmps_measure.argtypes = [C.c_void_p, C.c_uint32] + [P(C.c_double)] * 4
    lib.hmps_collapse_resample.argtypes = [C.c_void_p, C.c_int32,
                                           P(C.c_uint8)]
    lib.hmps_stats.argtypes = [C.c_void_p, P(hmps_stats_t)]
    lib.hmps_bond_dims.argtypes = [C.c_void_p, P(C.c_int32)]
    lib.hmps_measure_pairs.argtypes = [C.c_void_p, C.c_int32, P(C.c_int32),
                                       P(C.c_int32), P(C.c_double)]
    lib.hmps_susceptibility.argtypes = [C.c_void_p, C.c_double, C.c_int32,
                                        P(C.c_int32), P(C.c_double)]
    lib.hmps_svd_probe.argtypes = [C.c_void_p, C.c_int32, C.c_int32,
                                   P(C.c_double), C.c_int32, C.c_double,
                                   P(C.c_double), P(C.c_int32),
                                   P(C.c_double), P(C.c_double)]
    lib.hmps_read_site.argtypes = [C.c_void_p, C.c_int32, C.c_int32,
                                   P(C.c_double)]
    lib.hmps_load_bond.argtypes = [C.c_void_p] + [C.c_int32] * 4 + [
        P(C.c_double), P(C.c_double)]
    lib.hmps_apply_gate.argtypes = [C.c_void_p, C.c_double, C.c_double,
                                    C.c_int32, C.c_double, P(C.c_double)]
    lib.hmps_moments_reset.argtypes = [C.c_void_p]
    lib.hmps_bond_moments.argtypes = [C.c_void_p, P(C.c_int64),
                                      P(C.c_double), P(C.c_double),
                                      P(C.c_double)]
    lib.hmps_svd_probe_noalloc.argtypes = [
        C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
        C.c_double, C.c_void_p, P(C.c_int32), C.c_void_p, C.c_void_p]
    lib.hmps_svd_probe_noalloc.restype = C.c_int32
    lib.hmps_destroy.argtypes = [C.c_void_p]
    lib.hmps_destroy.restype = None
    lib.hmps_last_error.argtypes = [C.c_void_p]
    lib.hmps_last_error.restype = C.c_char_p
    lib.hmps_gate.argtypes = [C.c_double, C.c_double, P(C.c_double)]
    lib.hmps_schedule.argtypes = [P(hmps_lattice), P(C.c_int32),
                                  P(C.c_int32), P(C.c_int32), P(C.c_int32),
                                  C.c_int32]
    for name in ("hmps_create", "hmps_init_cluster_env", "hmps_evolve",
                 "hmps_measure", "hmps_collapse_resample", "hmps_stats",
                 "hmps_bond_dims", "hmps_gate", "hmps_schedule",
                 "hmps_svd_probe", "hmps_measure_pairs",
                 "hmps_susceptibility", "hmps_read_site", "hmps_load_bond",
                 "hmps_apply_gate", "hmps_init_cluster_env_at",
                 "hmps_evolve_updates", "hmps_last_spectrum",
                 "hmps_bond_charges", "hmps_set_width_rule"):
        getattr(lib, name).restype = C.c_int32
    _lib = lib
    return lib


class HmpsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hmps status {status}: {msg}")
        self.status = status


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


class Lattice:
    """Host arrays of an hmps_lattice kept alive with the struct."""

    def __init__(self, n_phys, bonds, order, in_cluster):
        self.n_phys = int(n_phys)
        self.bi = np.ascontiguousarray([b[0] for b in bonds], dtype=np.int32)
        self.bj = np.ascontiguousarray([b[1] for b in bonds], dtype=np.int32)
        self.bJ = np.ascontiguousarray([b[2] for b in bonds],
                                       dtype=np.float64)
        self.order = np.ascontiguousarray(order, dtype=np.int32)
        self.in_cluster = np.ascontiguousarray(in_cluster, dtype=np.uint8)
        self.n_bonds = len(bonds)
        self.c = hmps_lattice(self.n_phys, self.n_bonds,
                              _ptr(self.bi, C.c_int32),
                              _ptr(self.bj, C.c_int32),
                              _ptr(self.bJ, C.c_double),
                              _ptr(self.order, C.c_int32),
                              _ptr(self.in_cluster, C.c_uint8))


def hmps_workspace_bytes(max_chains, max_sites, chi_cap, max_bonds) -> int:
    return int(load().hmps_workspace_bytes(max_chains, max_sites, chi_cap,
                                           max_bonds))


def hmps_workspace_bytes_sym(max_chains, max_sites, chi_cap, max_bonds,
                             symmetry, max_blocks=0) -> int:
    return int(load().hmps_workspace_bytes_sym(max_chains, max_sites, chi_cap,
                                               max_bonds, symmetry,
                                               max_blocks))


def hmps_gate(J: float, x: float) -> np.ndarray:
    out = np.zeros(81)
    st = load().hmps_gate(J, x, _ptr(out, C.c_double))
    if st:
        raise HmpsError(st, "hmps_gate")
    return out.reshape(9, 9)


def hmps_schedule(lat: Lattice):
    """(n_sites, [(k, op)] of one Trotter step)."""
    lib = load()
    ns, nu = C.c_int32(), C.c_int32()
    st = lib.hmps_schedule(C.byref(lat.c), C.byref(ns), C.byref(nu), None,
                           None, 0)
    if st:
        raise HmpsError(st, "hmps_schedule")
    k = np.zeros(nu.value, np.int32)
    op = np.zeros(nu.value, np.int32)
    st = lib.hmps_schedule(C.byref(lat.c), C.byref(ns), C.byref(nu),
                           _ptr(k, C.c_int32), _ptr(op, C.c_int32), nu.value)
    if st:
        raise HmpsError(st, "hmps_schedule")
    return ns.value, list(zip(k.tolist(), op.tolist()))


class Context:
    """One hmps context with a torch-owned device workspace."""

    def __init__(self, max_chains, max_sites, chi_cap, max_bonds,
                 precision=PREC_FP64, device=0, stream=None, max_sweeps=0,
                 jacobi_tol=0.0, progress=None, symmetry=SYM_NONE,
                 max_blocks=0, width_rule=None):
        import torch
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("hmps needs a ROCm GPU (torch.cuda)")
        self.lib = lib
        self.device = device
        nbytes = hmps_workspace_bytes_sym(max_chains, max_sites, chi_cap,
                                          max_bonds, symmetry, max_blocks)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8,
                                     device=f"cuda:{device}")
        base = self.workspace.data_ptr()
        base = (base + 255) // 256 * 256
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        # progress(done, total) is called after every Trotter step
        self._progress = (PROGRESS_FN(lambda _u, d, t: progress(d, t))
                          if progress is not None else None)
        self.opt = hmps_options(device, C.c_void_p(stream.cuda_stream),
                                C.c_void_p(base), nbytes, max_chains,
                                max_sites, chi_cap, max_bonds, precision,
                                max_sweeps, jacobi_tol,
                                C.cast(self._progress, C.c_void_p)
                                if self._progress else None, None,
                                symmetry, max_blocks)
        h = C.c_void_p()
        st = lib.hmps_create(C.byref(h), C.byref(self.opt))
        if st:
            raise HmpsError(st, "hmps_create")
        self.h = h
        if width_rule is not None:
            self.hmps_set_width_rule(width_rule)
        self.n_chains = 0
        self.n_env = 0
        self.n_bonds = 0
        self.n_sites = 0

    def _check(self, st, what):
        if st:
            msg = self.lib.hmps_last_error(self.h).decode()
            raise HmpsError(st, f"{what}: {msg}")

    def hmps_init_cluster_env(self, lat: Lattice, n_chains: int, seed: int,
                              env_state=None, basis: int = 0,
                              chain_offset: int = 0, sample: int = 0):
        """hmps_init_cluster_env, or hmps_init_cluster_env_at when a chain
        offset or a start sample is given."""
        self._lat = lat
        es = None
        if env_state is not None:
            env_state = np.ascontiguousarray(env_state, dtype=np.uint8)
            es = _ptr(env_state, C.c_uint8)
        if chain_offset == 0 and sample == 0:
            st = self.lib.hmps_init_cluster_env(
                self.h, C.byref(lat.c), n_chains, C.c_uint64(seed), es, basis)
        else:
            st = self.lib.hmps_init_cluster_env_at(
                self.h, C.byref(lat.c), n_chains, C.c_uint64(seed),
                C.c_uint64(chain_offset), C.c_int64(sample), es, basis)
        self._check(st, "hmps_init_cluster_env")
        self.n_chains = n_chains
        self.n_bonds = lat.n_bonds
        s = self.hmps_stats()
        self.n_env = s.n_env
        self.n_sites = s.n_sites

    def hmps_evolve(self, beta, tau, chi_max, cutoff):
        self._check(self.lib.hmps_evolve(self.h, beta, tau, chi_max, cutoff),
                    "hmps_evolve")

    def hmps_evolve_updates(self, beta, tau, chi_max, cutoff, first, count):
        self._check(self.lib.hmps_evolve_updates(
            self.h, beta, tau, chi_max, cutoff, int(first), int(count)),
            "hmps_evolve_updates")

    def hmps_last_spectrum(self, cap):
        """(rank[n_chains], sigma[n_chains, cap]) of the last update."""
        rank = np.zeros(self.n_chains, np.int32)
        sig = np.zeros((self.n_chains, max(cap, 1)), np.float64)
        self._check(self.lib.hmps_last_spectrum(
            self.h, int(cap), _ptr(rank, C.c_int32), _ptr(sig, C.c_double)),
            "hmps_last_spectrum")
        return rank, sig[:, :cap]

    def hmps_measure(self, what=MEASURE_ALL):
        """Outputs whose bit is not in `what` come back as None."""
        B, nb = self.n_chains, self.n_bonds
        e, lw, qn = np.zeros(B), np.zeros(B), np.zeros(B)
        ss = np.zeros((B, max(nb, 1)))
        self._check(self.lib.hmps_measure(
            self.h, C.c_uint32(what), _ptr(e, C.c_double),
            _ptr(ss, C.c_double), _ptr(lw, C.c_double),
            _ptr(qn, C.c_double)), "hmps_measure")
        return {"energy": e if what & MEASURE_ENERGY else None,
                "bond_ss": ss[:, :nb] if what & MEASURE_BONDS else None,
                "logw": lw if what & MEASURE_LOGW else None,
                "qn": qn if what & MEASURE_QN else None}

    def hmps_moments_reset(self):
        self._check(self.lib.hmps_moments_reset(self.h), "hmps_moments_reset")

    def hmps_bond_moments(self):
        """Sample moments accumulated by hmps_measure(... |
        MEASURE_ACCUMULATE): count, per-bond mean and variance, energy mean
        and variance."""
        nb = self.n_bonds
        n = C.c_int64(0)
        mean, var = np.zeros(max(nb, 1)), np.zeros(max(nb, 1))
        emv = np.zeros(2)
        self._check(self.lib.hmps_bond_moments(
            self.h, C.byref(n), _ptr(mean, C.c_double), _ptr(var, C.c_double),
            _ptr(emv, C.c_double)), "hmps_bond_moments")
        return {"n": int(n.value), "mean": mean[:nb], "var": var[:nb],
                "energy_mean": float(emv[0]), "energy_var": float(emv[1])}

    def hmps_collapse_resample(self, basis: int):
        out = np.zeros((self.n_chains, max(self.n_env, 1)), np.uint8)
        self._check(self.lib.hmps_collapse_resample(
            self.h, basis, _ptr(out, C.c_uint8)), "hmps_collapse_resample")
        return out[:, : self.n_env]

    def hmps_stats(self):
        s = hmps_stats_t()
        self._check(self.lib.hmps_stats(self.h, C.byref(s)), "hmps_stats")
        return s

    def hmps_set_width_rule(self, rule):
        """rule: [(nvec_min, chains_min), ...] (see hmps_set_width_rule);
        [] restores the default."""
        nv = np.ascontiguousarray([r[0] for r in rule], np.int32)
        ch = np.ascontiguousarray([r[1] for r in rule], np.int32)
        self._check(self.lib.hmps_set_width_rule(
            self.h, len(rule), _ptr(nv, C.c_int32) if len(rule) else None,
            _ptr(ch, C.c_int32) if len(rule) else None),
            "hmps_set_width_rule")

    def hmps_bond_charges(self, chain, bond):
        """Charges of the indices of bond `bond` of chain `chain` (U(1))."""
        n = int(self.hmps_bond_dims()[chain, bond])
        out = np.zeros(max(n, 1), np.int32)
        self._check(self.lib.hmps_bond_charges(self.h, chain, bond,
                                               _ptr(out, C.c_int32)),
                    "hmps_bond_charges")
        return out[:n]

    def hmps_bond_dims(self):
        out = np.zeros((self.n_chains, self.n_sites + 1), np.int32)
        self._check(self.lib.hmps_bond_dims(self.h, _ptr(out, C.c_int32)),
                    "hmps_bond_dims")
        return out

    def hmps_measure_pairs(self, pairs):
        """<S_i.S_j> for physical-site pairs [(i, j)]: array [n_chains,
        n_pairs]."""
        pairs = np.asarray(pairs, np.int32).reshape(-1, 2)
        si = np.ascontiguousarray(pairs[:, 0])
        sj = np.ascontiguousarray(pairs[:, 1])
        out = np.zeros((self.n_chains, len(pairs)), np.float64)
        self._check(self.lib.hmps_measure_pairs(
            self.h, len(pairs), _ptr(si, C.c_int32), _ptr(sj, C.c_int32),
            _ptr(out, C.c_double)), "hmps_measure_pairs")
        return out

    def hmps_susceptibility(self, beta, center):
        """(beta/3) mean over j in center of sum_i <S_j.S_i>, per chain."""
        center = np.ascontiguousarray(center, np.int32)
        out = np.zeros(self.n_chains, np.float64)
        self._check(self.lib.hmps_susceptibility(
            self.h, float(beta), len(center), _ptr(center, C.c_int32),
            _ptr(out, C.c_double)), "hmps_susceptibility")
        return out

    def hmps_svd_probe(self, theta, chi_max, cutoff):
        """Truncated SVD of one update applied to theta' (m x n, m and n
        multiples of 3) on the device.  Returns (sigma[k], left[3, chi_l,
        k], right[3, k, chi_r]).  Replaces the context's chains."""
        theta = np.ascontiguousarray(theta, np.float64)
        m, n = theta.shape
        if m % 3 or n % 3:
            raise ValueError("theta dimensions must be multiples of 3")
        chi_l, chi_r = m // 3, n // 3
        kmax = min(m, n)
        sigma = np.zeros(kmax, np.float64)
        left = np.zeros(3 * chi_l * kmax, np.float64)
        right = np.zeros(3 * kmax * chi_r, np.float64)
        rank = C.c_int32(0)
        self._check(self.lib.hmps_svd_probe(
            self.h, chi_l, chi_r, _ptr(theta, C.c_double), int(chi_max),
            float(cutoff), _ptr(sigma, C.c_double), C.byref(rank),
            _ptr(left, C.c_double), _ptr(right, C.c_double)),
            "hmps_svd_probe")
        k = rank.value
        self.n_chains, self.n_sites = 1, 2
        return (sigma[:k].copy(), left[:3 * chi_l * k].reshape(3, chi_l, k),
                right[:3 * k * chi_r].reshape(3, k, chi_r))

    def hmps_read_site(self, chain, site):
        """Site tensor T[s, a, b] of one chain."""
        chi = self.hmps_bond_dims()[chain]
        out = np.zeros((3, int(chi[site]), int(chi[site + 1])), np.float64)
        self._check(self.lib.hmps_read_site(self.h, int(chain), int(site),
                                            _ptr(out, C.c_double)),
                    "hmps_read_site")
        return out

    def hmps_load_bond(self, center, right):
        """Replaces the chains by two-site segments: center [B, 3, chi_l,
        chi_m] (orthogonality centre) and right [B, 3, chi_m, chi_r]
        (right-orthonormal), layout T[s, a, b]."""
        center = np.ascontiguousarray(center, np.float64)
        right = np.ascontiguousarray(right, np.float64)
        if center.ndim != 4 or right.ndim != 4 or center.shape[1] != 3 or \
                right.shape[1] != 3 or center.shape[0] != right.shape[0] or \
                center.shape[3] != right.shape[2]:
            raise ValueError("center [B, 3, chi_l, chi_m] and right "
                             "[B, 3, chi_m, chi_r] expected")
        B, _, chi_l, chi_m = center.shape
        chi_r = right.shape[3]
        self._check(self.lib.hmps_load_bond(
            self.h, B, chi_l, chi_m, chi_r, _ptr(center, C.c_double),
            _ptr(right, C.c_double)), "hmps_load_bond")
        self.n_chains, self.n_sites = B, 2
        self.n_env = self.n_bonds = 0

    def hmps_apply_gate(self, J, x, chi_max, cutoff, want_logw=False):
        """One application of exp(-x J S.S) with its truncated SVD on the
        loaded bond of every chain; returns the log-weights if asked."""
        logw = np.zeros(self.n_chains, np.float64) if want_logw else None
        self._check(self.lib.hmps_apply_gate(
            self.h, float(J), float(x), int(chi_max), float(cutoff),
            _ptr(logw, C.c_double) if want_logw else None),
            "hmps_apply_gate")
        return logw

    def hmps_destroy(self):
        if getattr(self, "h", None):
            self.lib.hmps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.hmps_destroy()
        except Exception:
            pass
