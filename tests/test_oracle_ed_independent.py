"""The oracle's exact diagonalisation (thermal and ground-state energies of
the S=1 two-leg ladder, Results section) against a second, independent
brute force written here: the Hamiltonian is built sector by sector in
total S^z, from the action of S_i.S_j = S^z_i S^z_j + (S^+_i S^-_j +
S^-_i S^+_j)/2 on basis states (no Kronecker products, no code shared with
the oracle), and the ladder geometry is taken from (column, leg)
coordinates directly.  A wrong bond list, coupling assignment or spin-1
matrix element in either would show up as a different spectrum."""
import itertools
import math

import numpy as np
import pytest

from oracle import exact, model


def ladder_bonds(L, J_leg, J_rung):
    site = {(c, l): 2 * c + l for c in range(L) for l in range(2)}
    bonds = [(site[c, 0], site[c, 1], J_rung) for c in range(L)]
    bonds += [(site[c, l], site[c + 1, l], J_leg)
              for c in range(L - 1) for l in range(2)]
    return 2 * L, bonds


def raise_amp(m):
    # S^+ |1, m> = sqrt(s(s+1) - m(m+1)) |1, m+1>, s = 1
    return math.sqrt(2 - m * (m + 1)) if m < 1 else 0.0


def lower_amp(m):
    return math.sqrt(2 - m * (m - 1)) if m > -1 else 0.0


def spectrum(n, bonds):
    states = list(itertools.product((1, 0, -1), repeat=n))
    sectors = {}
    for st in states:
        sectors.setdefault(sum(st), []).append(st)
    energies = []
    for mz, basis in sectors.items():
        index = {st: i for i, st in enumerate(basis)}
        H = np.zeros((len(basis), len(basis)))
        for col, st in enumerate(basis):
            for i, j, J in bonds:
                H[col, col] += J * st[i] * st[j]
                for up, dn in ((i, j), (j, i)):
                    amp = raise_amp(st[up]) * lower_amp(st[dn])
                    if amp == 0.0:
                        continue
                    new = list(st)
                    new[up] += 1
                    new[dn] -= 1
                    H[index[tuple(new)], col] += 0.5 * J * amp
        assert np.allclose(H, H.T)
        energies.extend(np.linalg.eigvalsh(H))
    return np.sort(np.array(energies))


def thermal(e, beta):
    w = np.exp(-beta * (e - e.min()))
    return float((w * e).sum() / w.sum())


@pytest.mark.parametrize("J_rung", [1.0, 0.5])
def test_ladder_2x3_energies_match_an_independent_diagonalisation(J_rung):
    n, bonds = ladder_bonds(3, 1.0, J_rung)
    e = spectrum(n, bonds)
    assert len(e) == 3 ** n
    lat = model.ladder(3, 1.0, J_rung, W=0)
    for beta in (0.5, 1.0, 2.0, 5.0):
        want = thermal(e, beta)
        got = exact.thermal_energy(lat, beta)
        assert abs(got - want) <= 1e-12 * abs(want), (beta, got, want)
    assert abs(exact.ground_energy(lat) - e[0]) <= 1e-12 * abs(e[0])


def test_spectrum_of_one_bond():
    # S_1.S_2 = (S(S+1) - 4)/2 on total spin S = 0, 1, 2: -2, -1 (x3), 1 (x5)
    e = spectrum(2, [(0, 1, 1.0)])
    want = np.array([-2.0] + [-1.0] * 3 + [1.0] * 5)
    assert np.abs(e - want).max() < 1e-14
