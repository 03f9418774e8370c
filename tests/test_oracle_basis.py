"""Pins for the symmetry-adapted bases and the block Hamiltonians (Sec. II A, App. A)."""
from math import comb

import numpy as np
import pytest
import scipy.sparse as sp

import qoc_workloads as W
from oracle import basis, counts, grape, groups, pauli


def _all_columns(n, stride, refl, route):
    cols = []
    for lab in counts.irrep_labels(n // stride, refl):
        Vs = basis.projector_basis(n, lab, stride, refl) if route == "projector" else \
            basis.convention_basis(n, lab, stride, refl)[0]
        cols += Vs
    return np.concatenate(cols, axis=1)


@pytest.mark.parametrize("route", ["projector", "convention"])
@pytest.mark.parametrize("n,stride,refl", [(5, 1, True), (6, 1, True), (8, 2, True), (6, 1, False), (8, 1, True)])
def test_adjoint_matrix_is_unitary(n, stride, refl, route):
    A = _all_columns(n, stride, refl, route)
    assert A.shape == (2 ** n, 2 ** n)
    assert np.abs(A.conj().T @ A - np.eye(2 ** n)).max() < 1e-12


def _heis_terms(n):
    return W.heisenberg_ring_terms(0.83, 0.37) + [W.ring_pair(0.21, "zz", 2 if n >= 5 else 1)]


@pytest.mark.parametrize("route", ["projector", "convention"])
@pytest.mark.parametrize("n", [4, 6, 7])
def test_block_diagonal_and_spectrum_union(n, route):
    terms = _heis_terms(n) + [W.one_body(0.4, "x"), W.one_body(-0.3, "y")]
    H = pauli.hamiltonian(n, terms).toarray()
    blocks = grape.block_system(n, terms, [], "dihedral", 1, route)
    evs = []
    for b in blocks:
        for V in b["V"]:
            Hb = V.conj().T @ H @ V
            # leak residual: H V = V (V^dag H V) exactly when span(V) is invariant
            assert np.linalg.norm(H @ V - V @ Hb) <= 1e-13 * np.linalg.norm(H)
            # both copies carry the same block (transfer operator / reflection copy)
            assert np.abs(Hb - b["H0"]).max() < 1e-12
            evs.append(np.linalg.eigvalsh(Hb))
    assert np.allclose(np.sort(np.concatenate(evs)), np.linalg.eigvalsh(H), atol=1e-11)


@pytest.mark.parametrize("n", [5, 6, 8])
def test_first_block_canonical_entries(n):
    """The A1 block is canonical: both routes give identical entries, and they equal
    sqrt(|O_a|/|O_b|) * sum_{y in O_b} H[y, a] over representatives a, b."""
    terms = _heis_terms(n) + [W.one_body(0.7, "x"), W.one_body(0.2, "y")]
    H = pauli.hamiltonian(n, terms).toarray()
    bp = grape.block_system(n, terms, [], "dihedral", 1, "projector")[0]
    bc = grape.block_system(n, terms, [], "dihedral", 1, "convention")[0]
    assert np.abs(bp["H0"] - bc["H0"]).max() < 1e-12
    G = groups.ring_group(n)
    imgs = basis.all_images(n, G)
    reps = bc["reps"]
    orbit = {a: np.unique(imgs[:, a]) for a in reps}
    for i, b in enumerate(reps):
        for j, a in enumerate(reps):
            val = np.sqrt(len(orbit[a]) / len(orbit[b])) * H[orbit[b], a].sum()
            assert abs(bc["H0"][i, j] - val) < 1e-12


@pytest.mark.parametrize("n", [3, 4, 6])
def test_paper_structure_statements(n):
    """Sec. II A: A^dag H_z A stays diagonal; all-up and all-down lie in the first subspace;
    H_x, H_y, H_z are invariant under every qubit permutation; H_z,cpl only under D_n (n >= 4)."""
    Hz = pauli.hamiltonian(n, [W.one_body(1.0, "z")]).toarray()
    for b in grape.block_system(n, [W.one_body(1.0, "z")], [], "dihedral", 1, "projector"):
        assert np.abs(b["H0"] - np.diag(np.diag(b["H0"]))).max() < 1e-12
    A1 = basis.projector_basis(n, "A1")[0]
    for x in (0, 2 ** n - 1):
        e = np.zeros(2 ** n)
        e[x] = 1
        assert np.linalg.norm(A1 @ (A1.conj().T @ e) - e) < 1e-12
    swap = np.arange(n)
    swap[[0, 1]] = [1, 0]
    P = groups.operator(swap, n)
    for a in "xyz":
        Ha = pauli.hamiltonian(n, [W.one_body(1.0, a)]).toarray()
        assert np.abs(P @ Ha - Ha @ P).max() == 0.0
    Hc = pauli.hamiltonian(n, [W.ring_pair(1.0, "zz")]).toarray()
    for (l, f), perm in groups.ring_group(n):
        U = groups.operator(perm, n)
        assert np.abs(U @ Hc - Hc @ U).max() == 0.0
    comm = np.abs(P @ Hc - Hc @ P).max()
    assert (comm == 0.0) if n == 3 else (comm > 0.5)


def test_staggered_controls_need_two_site_rotation():
    """Staggered sigma_z and even-qubit sigma_x break the one-site rotation but keep
    the two-site rotation and the site-centred reflection."""
    n = 6
    for t in ([W.one_body(1.0, "z", stagger=True)], [W.one_body(1.0, "x", sites="even")]):
        H = pauli.hamiltonian(n, t).toarray()
        for (l, f), expect in [((1, 0), False), ((2, 0), True), ((0, 1), True), ((2, 1), True)]:
            U = groups.operator(groups.element(n, 1, l, f), n)
            ok = np.abs(U @ H - H @ U).max() == 0.0
            assert ok == expect


def _dicke(n, w):
    v = np.zeros(2 ** n)
    for x in range(2 ** n):
        if bin(x).count("1") == w:
            v[x] = 1.0
    return v / np.sqrt(comb(n, w))


@pytest.mark.parametrize("n", [3, 4, 6])
def test_sn_top_block_equals_dicke_projection(n):
    """J = n/2 block of the closed form equals the Hamiltonian projected on the Dicke
    states |n, w> (symmetric subspace), w = number of down spins."""
    terms = [W.one_body(0.9, "z"), W.one_body(0.4, "x"), W.one_body(-0.25, "y"),
             W.all_pairs(0.3, "xx"), W.all_pairs(-0.6, "zz")]
    H = pauli.hamiltonian(n, terms).toarray()
    D = np.stack([_dicke(n, w) for w in range(n + 1)], axis=1)
    Hd = D.T @ H @ D
    twoJ, Hb = basis.sn_blocks(n, terms)[0]
    # |J, M> with M = J - w has w down spins; the closed form's phase convention is the
    # Condon-Shortley one, which for these real symmetric sums is the plain Dicke basis
    assert twoJ == n
    assert np.abs(Hb - Hd).max() < 1e-12


@pytest.mark.parametrize("n", [4, 5, 7])
def test_sn_spectrum_union(n):
    terms = [W.one_body(0.9, "z"), W.one_body(0.4, "x"), W.all_pairs(0.3, "xx"), W.all_pairs(-0.2, "yy")]
    H = pauli.hamiltonian(n, terms).toarray()
    evs = []
    for (twoJ, Hb), (_, size, mult) in zip(basis.sn_blocks(n, terms), counts.sn_sectors(n)):
        assert Hb.shape[0] == size
        evs += list(np.linalg.eigvalsh(Hb)) * mult
    assert np.allclose(np.sort(evs), np.linalg.eigvalsh(H), atol=1e-11)
