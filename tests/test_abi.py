"""Host-side checks of the C ABI library (no GPU needed): it loads, it
exports every function include/hmps.h declares, and its host-only helpers
(update list, gate) agree with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg

from oracle import exact, model
from paper_1910_09142_amd import hmps, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hmps.h")).read()
    return sorted(set(re.findall(r"\b(hmps_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = hmps.load()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(hmps.EXPORTS)


@pytest.mark.parametrize("L,W,Jr", [(1, 1, 1.0), (3, 1, 1.0), (8, 2, 1.0),
                                    (16, 2, 0.5), (32, 4, 1.0), (4, 0, 0.5),
                                    (4, 4, 1.0)])
def test_schedule_matches_oracle(L, W, Jr):
    n, bonds, order, mask = workloads.ladder_arrays(L, 1.0, Jr, W)
    olat = model.ladder(L, 1.0, Jr, W=W)
    assert (olat.bonds, olat.order) == (bonds, order)
    assert [int(x) for x in olat.in_cluster] == mask
    ns, ups = hmps.hmps_schedule(hmps.Lattice(n, bonds, order, mask))
    sch = model.schedule(olat)
    assert ns == model.layout(olat).length
    assert ups == [(k, op) for (k, op) in sch.step]


@pytest.mark.parametrize("L,sites", [(3, {0, 3, 4}), (4, {0, 1, 4, 5}),
                                     (6, {1, 2, 7, 8, 11}), (5, set())])
def test_schedule_matches_oracle_for_any_cluster_mask(L, sites):
    # checkerboard / interleaved / scattered purified sites
    base = model.ladder(L, 1.0, 1.0, W=0)
    mask = [int(i in sites) for i in range(base.n_phys)]
    olat = model.Lattice(base.n_phys, base.bonds, base.order,
                         [bool(m) for m in mask])
    ns, ups = hmps.hmps_schedule(hmps.Lattice(base.n_phys, base.bonds,
                                              base.order, mask))
    lay = model.layout(olat)
    assert ns == lay.length == base.n_phys + len(sites)
    assert ups == [(k, op) for (k, op) in model.schedule(olat).step]


@pytest.mark.parametrize("J,x", [(1.0, 0.025), (0.5, 0.05), (2.0, 0.3)])
def test_gate_matches_expm(J, x):
    h = exact.bond_operator(0, 1, 2)
    assert np.abs(hmps.hmps_gate(J, x) - scipy.linalg.expm(-x * J * h)).max() < 1e-14


def test_invalid_lattices_rejected():
    bad = [
        hmps.Lattice(2, [(0, 0, 1.0)], [0, 1], [0, 0]),      # self bond
        hmps.Lattice(2, [(0, 2, 1.0)], [0, 1], [0, 0]),      # out of range
        hmps.Lattice(2, [(0, 1, 1.0)], [0, 0], [0, 0]),      # not a permutation
        hmps.Lattice(2, [(0, 1, float("nan"))], [0, 1], [0, 0]),
    ]
    for lat in bad:
        with pytest.raises(hmps.HmpsError) as e:
            hmps.hmps_schedule(lat)
        assert e.value.status == hmps.HMPS_E_INVALID


def test_workspace_bytes_grows_with_capacity():
    a = hmps.hmps_workspace_bytes(1, 8, 32, 7)
    b = hmps.hmps_workspace_bytes(2, 8, 32, 7)
    c = hmps.hmps_workspace_bytes(1, 8, 64, 7)
    assert 0 < a < b and a < c
    assert hmps.hmps_workspace_bytes(0, 8, 32, 7) == 0


def test_create_rejects_bad_options_without_gpu():
    lib = hmps.load()
    h = ctypes.c_void_p()
    opt = hmps.hmps_options(0, None, None, 0, 0, 8, 32, 7, 0, 0, 0.0, None, None)
    assert lib.hmps_create(ctypes.byref(h), ctypes.byref(opt)) == hmps.HMPS_E_INVALID
    opt = hmps.hmps_options(0, None, None, 0, 1, 8, 32, 7, 0, 0, 0.0, None, None)
    assert lib.hmps_create(ctypes.byref(h), ctypes.byref(opt)) == hmps.HMPS_E_NOMEM
    # chains run along a grid dimension of at most 65535 blocks
    opt = hmps.hmps_options(0, None, None, 0, 65536, 8, 32, 7, 0, 0, 0.0, None,
                            None)
    assert lib.hmps_create(ctypes.byref(h), ctypes.byref(opt)) == hmps.HMPS_E_INVALID
    opt = hmps.hmps_options(0, None, None, 0, 1, 8, 641, 7, 0, 0, 0.0, None, None)
    assert lib.hmps_create(ctypes.byref(h), ctypes.byref(opt)) == hmps.HMPS_E_INVALID
    opt = hmps.hmps_options(0, None, None, 0, 1, 8, 32, 7, 2, 0, 0.0, None, None)
    assert lib.hmps_create(ctypes.byref(h), ctypes.byref(opt)) == hmps.HMPS_E_INVALID
