"""Closed-form counts that pin the basis construction (Table I; App. A).

* necklaces / bracelets: number of orbits of n-bit strings under C_n / D_n,
  by Burnside's lemma with Euler's totient; the D_n first-subspace dimension of
  Table I is the number of D_n orbits (each orbit contributes one orbit sum).
* block sizes from characters: the multiplicity of irrep theta in the
  permutation representation on C^{2^n} is (1/|G|) sum_g conj(chi_theta(g)) tr(U_g),
  and tr(U_g) = 2^{#cycles of g} because a basis state is fixed exactly when
  it is constant on every cycle.
* S_n: the J sector of n spin-1/2 has dimension 2J+1 and multiplicity
  C(n, n/2-J) - C(n, n/2-J-1)  (Clebsch-Gordan route of App. A).
"""
from __future__ import annotations

from fractions import Fraction
from math import comb, gcd

import numpy as np

from . import groups


def totient(n: int) -> int:
    return sum(1 for k in range(1, n + 1) if gcd(k, n) == 1)


def necklaces(n: int) -> int:
    return sum(totient(d) * 2 ** (n // d) for d in range(1, n + 1) if n % d == 0) // n


def bracelets(n: int) -> int:
    if n % 2 == 0:
        return necklaces(n) // 2 + 3 * 2 ** (n // 2) // 4
    return necklaces(n) // 2 + 2 ** ((n - 1) // 2)


def cycles(perm) -> int:
    perm = list(perm)
    seen = [False] * len(perm)
    c = 0
    for i in range(len(perm)):
        if not seen[i]:
            c += 1
            j = i
            while not seen[j]:
                seen[j] = True
                j = perm[j]
    return c


def irrep_labels(L: int, reflection: bool = True):
    """Irreps in the library's block order: A1, A2, (B1, B2 when L even), E_1.. ; or k_0..k_{L-1}."""
    if not reflection:
        return [f"k{m}" for m in range(L)]
    labs = ["A1", "A2"]
    if L % 2 == 0:
        labs += ["B1", "B2"]
    nE = (L - 1) // 2 if L % 2 else L // 2 - 1
    labs += [f"E{m}" for m in range(1, nE + 1)]
    return labs


def character(label: str, L: int, l: int, f: int):
    """Character of rho^l phi^f.  B1 has chi(rho) = -1 and chi(phi) = +1 for the
    site-centred reflection phi; E_m has the 2x2 rotation/reflection matrices."""
    if label == "A1":
        return 1.0
    if label == "A2":
        return -1.0 if f else 1.0
    if label == "B1":
        return float((-1) ** l)
    if label == "B2":
        return float((-1) ** l) * (-1.0 if f else 1.0)
    if label.startswith("E"):
        m = int(label[1:])
        return 0.0 if f else 2.0 * np.cos(2 * np.pi * m * l / L)
    if label.startswith("k"):
        m = int(label[1:])
        return np.exp(2j * np.pi * m * l / L)
    raise ValueError(label)


def irrep_dim(label: str) -> int:
    return 2 if label.startswith("E") else 1


def block_sizes(n: int, stride: int = 1, reflection: bool = True):
    """{label: (m_theta, d_theta)} from the character formula."""
    L = n // stride
    G = groups.ring_group(n, stride, reflection)
    out = {}
    for lab in irrep_labels(L, reflection):
        tot = 0.0 + 0.0j
        for (l, f), perm in G:
            tot += np.conj(character(lab, L, l, f)) * 2 ** cycles(perm)
        m = tot / len(G)
        mi = int(round(m.real))
        if abs(m - mi) > 1e-6:
            raise AssertionError("non-integer multiplicity")
        out[lab] = (mi, irrep_dim(lab))
    return out


def sn_sectors(n: int):
    """[(J (as Fraction), size 2J+1, multiplicity)] for J = n/2, n/2-1, ..., exact integers."""
    out = []
    twoJ = n
    while twoJ >= 0:
        k = (n - twoJ) // 2
        mult = comb(n, k) - (comb(n, k - 1) if k >= 1 else 0)
        out.append((Fraction(twoJ, 2), twoJ + 1, mult))
        twoJ -= 2
    return out
