"""Pins for orbit enumeration and block sizes (Table I; App. A)."""
import os
from math import comb

import numpy as np
import pytest

from oracle import basis, counts, groups

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_dims.txt")


def table1():
    rows = []
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            rows.append(tuple(int(v) for v in line.split()))
    return rows


@pytest.mark.parametrize("row", table1())
def test_table1_dihedral_first_block(row):
    n, dimH, dimS, dimD = row
    assert dimH == 2 ** n
    # bracelet count by Burnside, the A1 multiplicity by characters, and brute-force orbits
    assert counts.bracelets(n) == dimD
    assert counts.block_sizes(n)["A1"][0] == dimD
    if n <= 12:
        reps, _ = basis.orbit_reps(n)
        assert len(reps) == dimD


@pytest.mark.parametrize("row", table1())
def test_table1_symmetric_first_block(row):
    n, _, dimS, _ = row
    J, size, mult = counts.sn_sectors(n)[0]
    assert size == dimS and mult == 1


def _orbits_by_closure(n, gens):
    """Orbits by breadth-first closure under the generators only (pure Python)."""
    seen = {}
    reps = []
    for x in range(2 ** n):
        if x in seen:
            continue
        orbit = {x}
        frontier = [x]
        while frontier:
            y = frontier.pop()
            for g in gens:
                z = 0
                for p in range(n):
                    if (y >> p) & 1:
                        z |= 1 << int(g[p])
                if z not in orbit:
                    orbit.add(z)
                    frontier.append(z)
        for y in orbit:
            seen[y] = min(orbit)
        reps.append(min(orbit))
    return sorted(reps)


@pytest.mark.parametrize("n,stride,refl", [(3, 1, True), (5, 1, True), (6, 1, True), (7, 1, False),
                                           (8, 1, True), (8, 2, True), (9, 3, True), (10, 1, False)])
def test_orbits_match_generator_closure(n, stride, refl):
    gens = [groups.element(n, stride, 1, 0)] + ([groups.element(n, stride, 0, 1)] if refl else [])
    reps, sizes = basis.orbit_reps(n, stride, refl)
    assert list(reps) == _orbits_by_closure(n, gens)
    L = n // stride
    assert sizes.sum() == 2 ** n
    assert all((2 * L if refl else L) % s == 0 for s in sizes)


@pytest.mark.parametrize("n", list(range(3, 17)))
def test_necklace_count(n):
    if n <= 12:
        reps, _ = basis.orbit_reps(n, 1, False)
        assert len(reps) == counts.necklaces(n)
    assert counts.necklaces(n) >= counts.bracelets(n)


@pytest.mark.parametrize("n,stride", [(n, 1) for n in range(2, 17)] + [(14, 2), (12, 2), (12, 3), (12, 4)])
def test_block_sizes_sum(n, stride):
    for refl in (True, False):
        bs = counts.block_sizes(n, stride, refl)
        assert sum(m * d for m, d in bs.values()) == 2 ** n


def test_config4_group_sizes():
    bs = counts.block_sizes(14, 2, True)
    assert bs == {"A1": (1300, 1), "A2": (1044, 1), "E1": (2340, 2), "E2": (2340, 2), "E3": (2340, 2)}


@pytest.mark.parametrize("n", [3, 4, 7, 12, 31, 128])
def test_sn_multiplicities(n):
    secs = counts.sn_sectors(n)
    assert sum(size * mult for _, size, mult in secs) == 2 ** n
    assert len(secs) == n // 2 + 1
    # multiplicity of J = n/2 - k equals the number of standard Young tableaux of shape (n-k, k)
    for k, (_, _, mult) in enumerate(secs):
        assert mult == comb(n, k) * (n - 2 * k + 1) // (n - k + 1)


@pytest.mark.parametrize("n,stride,refl", [(6, 1, True), (8, 1, True), (8, 2, True), (6, 1, False), (9, 1, True)])
def test_basis_dimensions_match_characters(n, stride, refl):
    bs = counts.block_sizes(n, stride, refl)
    for lab, (m, d) in bs.items():
        Vp = basis.projector_basis(n, lab, stride, refl)
        Vc, _ = basis.convention_basis(n, lab, stride, refl)
        assert len(Vp) == d and len(Vc) == d
        for V in Vp + Vc:
            assert V.shape == (2 ** n, m)
