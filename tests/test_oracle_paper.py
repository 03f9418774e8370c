"""The paper's spectral statements on its Ising rings (Eqs. (5)-(7); Sec. III A)."""
import numpy as np
import pytest

import qoc_workloads as W
from oracle import grape


def _frequencies(n, h0_terms, tol=1e-9):
    """Distinct transition frequencies between first-subspace eigenstates of H0 that H_x connects."""
    blk = grape.block_system(n, h0_terms, [[W.one_body(0.5, "x")]], "dihedral", 1)[0]
    e, V = np.linalg.eigh(blk["H0"])
    Hx = V.conj().T @ blk["Hk"][0] @ V
    freqs = []
    for a in range(len(e)):
        for b in range(a + 1, len(e)):
            if abs(Hx[a, b]) > 1e-9 and abs(e[a] - e[b]) > tol:
                freqs.append(abs(e[a] - e[b]))
    freqs = np.sort(freqs)
    distinct = [f for i, f in enumerate(freqs) if i == 0 or f - freqs[i - 1] > 1e-7]
    return distinct


@pytest.mark.parametrize("n", [4, 6])
def test_no_coupling_one_frequency(n):
    """c_cpl = 0: equally spaced levels, one resonance frequency (the Zeeman splitting Bz)."""
    f = _frequencies(n, W.ising_ring_terms(1.3, 0.0))
    assert len(f) == 1 and abs(f[0] - 1.3) < 1e-12


@pytest.mark.parametrize("n", [3, 4, 9])
def test_nearest_neighbour_three_frequencies(n):
    """Nearest-neighbour coupling: three frequencies Bz - c, Bz, Bz + c for n >= 3... here
    in the Eq. (5) normalisation a single flip changes the wall term by 0 or +-c."""
    Bz, c = 1.0, 0.3
    f = _frequencies(n, W.ising_ring_terms(Bz, c))
    assert len(f) == 3
    assert np.allclose(f, [Bz - c, Bz, Bz + c])


def test_full_coupling_n4_six_frequencies():
    """Eq. (7) at n = 4 with generic couplings: six distinct resonance frequencies."""
    f = _frequencies(4, W.full_coupling_terms(4, 1.0, [0.3, 0.17]))
    assert len(f) == 6
