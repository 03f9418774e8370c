"""Symmetry-adapted bases (Sec. II A; App. A, Eqs. (A1)-(A2)).

Three independent constructions:

1. ``projector_basis``: the paper's route.  For each irrep theta with real
   orthogonal matrices A^theta(g), the group-algebra element
   O^theta_j = sum_g A^theta_jj(g) g (Eq. (A2)), normalised to the projector
   P^theta_jj = (d_theta/|G|) sum_g A^theta_jj(g) U_g, is applied to every Fock
   state of every orbit; an orthonormal basis of the span is kept (SVD, rank by
   tolerance).  For two-dimensional irreps the second row is obtained with the
   transfer operator P^theta_21 so that both copies carry identical blocks.
2. ``convention_basis``: the momentum/parity states that the library uses,
   written out by brute force from their definition:
     1-dim irrep chi, orbit representative a (minimum of its G-orbit), allowed
     when chi is trivial on the stabiliser of a:
        |a,chi> = |O_a|^{-1/2} sum_{y in O_a} conj(chi(g_y)) |y>,   g_y a = y;
     E_m (k = 2 pi m / L), cyclic representative c with period P_c, allowed
     when m P_c = 0 mod L:
        |c,k> = P_c^{-1/2} sum_{l<P_c} exp(-i k l) |rho^l c>,
     second copy U_phi |c,k>.
3. ``sn_block_operators``: the |J,M> closed form of the S_n decomposition
   (Clebsch-Gordan route named in App. A), M = J, J-1, ..., -J.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import counts, groups


# ----------------------------------------------------------------------------- orbits
def all_images(n: int, G):
    """Array (|G|, 2^n): images of every basis state under every group element."""
    x = np.arange(2 ** n, dtype=np.int64)
    return np.stack([groups.act(perm, x) for _, perm in G])


def orbit_reps(n: int, stride: int = 1, reflection: bool = True):
    """Sorted orbit representatives (minimum of each orbit) and orbit sizes, by brute force."""
    G = groups.ring_group(n, stride, reflection)
    imgs = all_images(n, G)
    rep = imgs.min(axis=0)
    reps = np.unique(rep)
    sizes = np.array([len(np.unique(imgs[:, a])) for a in reps])
    return reps, sizes


def irrep_matrix(label: str, L: int, l: int, f: int) -> np.ndarray:
    """Real orthogonal (or, for C_L, complex 1x1) irrep matrix of rho^l phi^f."""
    if label.startswith("E"):
        m = int(label[1:])
        a = 2 * np.pi * m * l / L
        R = np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])
        return R @ np.diag([1.0, -1.0]) if f else R
    return np.array([[counts.character(label, L, l, f)]])


# ----------------------------------------------------------------------------- route 1
def projector_basis(n: int, label: str, stride: int = 1, reflection: bool = True, tol=1e-9):
    """Isometry columns (2^n x m, and the second row's for 2-dim irreps) from Eq. (A2) projectors."""
    L = n // stride
    G = groups.ring_group(n, stride, reflection)
    imgs = all_images(n, G)
    d = counts.irrep_dim(label)
    mats = [irrep_matrix(label, L, l, f) for (l, f), _ in G]
    rep = imgs.min(axis=0)
    dim = 2 ** n
    cols = []
    for a in np.unique(rep):
        orbit = np.unique(imgs[:, a])
        pos = {int(y): i for i, y in enumerate(orbit)}
        M = np.zeros((len(orbit), len(orbit)), dtype=complex)
        for col, y in enumerate(orbit):
            for gi in range(len(G)):
                M[pos[int(imgs[gi, y])], col] += d / len(G) * np.conj(mats[gi][0, 0])
        U, s, _ = np.linalg.svd(M)
        r = int(np.sum(s > tol))
        for c in range(r):
            v = U[:, c]
            if label == "A1":
                v = v * (np.sign(v.sum().real) or 1.0)
            full = np.zeros(dim, dtype=complex)
            full[orbit] = v
            cols.append(full)
    V1 = np.array(cols).T if cols else np.zeros((dim, 0), dtype=complex)
    if d == 1:
        return [V1]
    # second row through the transfer operator P_21 = (d/|G|) sum_g conj(A_21(g)) U_g
    V2 = np.zeros_like(V1)
    for gi in range(len(G)):
        coef = d / len(G) * np.conj(mats[gi][1, 0])
        if coef != 0.0:
            V2[imgs[gi], :] += coef * V1
    return [V1, V2]


# ----------------------------------------------------------------------------- route 2
def _group_element_to(imgs, G, src, dst):
    """Index of some group element g with g.src = dst."""
    hits = np.nonzero(imgs[:, src] == dst)[0]
    return int(hits[0])


def convention_basis(n: int, label: str, stride: int = 1, reflection: bool = True):
    """(list of copies' isometries 2^n x m, list of representatives) in the library convention."""
    L = n // stride
    dim = 2 ** n
    G = groups.ring_group(n, stride, reflection)
    imgs = all_images(n, G)
    if label.startswith("E") or label.startswith("k"):
        m = int(label[1:])
        k = 2 * np.pi * m / L
        Gc = groups.ring_group(n, stride, False)
        cimgs = all_images(n, Gc)
        crep = cimgs.min(axis=0)
        cols, reps = [], []
        for c in np.unique(crep):
            P = next(l for l in range(1, L + 1) if cimgs[l % L, c] == c)
            if (m * P) % L:
                continue
            v = np.zeros(dim, dtype=complex)
            for l in range(P):
                v[cimgs[l, c]] += np.exp(-1j * k * l) / np.sqrt(P)
            cols.append(v)
            reps.append(int(c))
        V1 = np.array(cols).T if cols else np.zeros((dim, 0), dtype=complex)
        if label.startswith("k"):
            return [V1], reps
        phi = groups.element(n, stride, 0, 1)
        V2 = np.zeros_like(V1)
        V2[groups.act(phi, np.arange(dim)), :] = V1
        return [V1, V2], reps
    rep = imgs.min(axis=0)
    cols, reps = [], []
    for a in np.unique(rep):
        stab = [gi for gi in range(len(G)) if imgs[gi, a] == a]
        chis = [counts.character(label, L, *G[gi][0]) for gi in stab]
        if any(abs(c - 1.0) > 1e-12 for c in chis):
            continue
        orbit = np.unique(imgs[:, a])
        v = np.zeros(dim, dtype=complex)
        for y in orbit:
            gi = _group_element_to(imgs, G, a, y)
            v[y] = np.conj(counts.character(label, L, *G[gi][0])) / np.sqrt(len(orbit))
        cols.append(v)
        reps.append(int(a))
    V1 = np.array(cols).T if cols else np.zeros((dim, 0), dtype=complex)
    return [V1], reps


def project(H, V):
    """A^dagger H A for an isometry A = V (H sparse or dense)."""
    HV = H @ V
    return V.conj().T @ HV


# ----------------------------------------------------------------------------- S_n
def sn_collective(twoJ: int):
    """(2S_x, 2S_y, 2S_z) on the |J,M> basis, M = J, J-1, ..., -J, with J = twoJ/2."""
    J = twoJ / 2.0
    Ms = J - np.arange(twoJ + 1)
    Sp = np.zeros((twoJ + 1, twoJ + 1), dtype=complex)
    for r in range(1, twoJ + 1):
        M = Ms[r]  # S_+ |J,M> = sqrt(J(J+1) - M(M+1)) |J,M+1>, and M+1 sits at row r-1
        Sp[r - 1, r] = np.sqrt(J * (J + 1) - M * (M + 1))
    Sm = Sp.conj().T
    return Sp + Sm, -1j * (Sp - Sm), np.diag(2.0 * Ms).astype(complex)


def sn_term_block(n: int, twoJ: int, term: dict) -> np.ndarray:
    """Block of one S_n-invariant term in the J sector: sum_i sigma_a = 2 S_a and
    sum_{i<j} sigma_a^i sigma_a^j = ((2 S_a)^2 - n)/2."""
    S = dict(zip("xyz", sn_collective(twoJ)))
    c = term["coeff"]
    if term["kind"] == "one_body":
        if term["sites"] != "all" or term.get("stagger"):
            raise ValueError("one-body term is not S_n invariant")
        return c * S[term["op"]]
    if term["kind"] == "all_pairs" and term["op"][0] == term["op"][1]:
        T = S[term["op"][0]]
        return c * (T @ T - n * np.eye(twoJ + 1)) / 2.0
    raise ValueError("term is not S_n invariant")


def sn_blocks(n: int, terms):
    """[(twoJ, matrix)] for J = n/2, n/2-1, ...; one copy per J."""
    out = []
    twoJ = n
    while twoJ >= 0:
        H = np.zeros((twoJ + 1, twoJ + 1), dtype=complex)
        for t in terms:
            H = H + sn_term_block(n, twoJ, t)
        out.append((twoJ, H))
        twoJ -= 2
    return out
