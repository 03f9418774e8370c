"""Device orbit enumeration, block tables and state maps against the brute-force oracle
(App. A, Eq. (A2); Table I).  Integer results are compared bit for bit."""
import numpy as np
import pytest

from oracle import basis as obasis
from oracle import counts

pytestmark = pytest.mark.gpu

CASES = [(3, 1, True), (4, 1, True), (5, 1, True), (6, 1, True), (8, 1, True), (8, 2, True), (9, 3, True),
         (10, 1, False), (12, 1, True), (12, 4, True), (14, 2, True), (7, 7, True), (1, 1, True), (2, 1, True)]


def _group(refl):
    return "dihedral" if refl else "cyclic"


@pytest.mark.parametrize("n,stride,refl", CASES)
def test_orbits_bit_exact(lib, n, stride, refl):
    print(f"orbits n={n} stride={stride} refl={refl}", flush=True)
    B = lib.Basis(n, _group(refl), stride)
    reps, _ = obasis.orbit_reps(n, stride, refl)
    creps, _ = obasis.orbit_reps(n, stride, False)
    assert np.array_equal(B.reps(0), reps.astype(np.uint64))
    assert np.array_equal(B.reps(1), creps.astype(np.uint64))
    sizes = counts.block_sizes(n, stride, refl)
    labs = [l for l in counts.irrep_labels(n // stride, refl) if sizes[l][0] > 0]
    assert B.sizes == [sizes[l][0] for l in labs]
    assert B.copies == [sizes[l][1] for l in labs]
    if n <= 12:
        for b, lab in enumerate(labs):
            _, oreps = obasis.convention_basis(n, lab, stride, refl)
            assert np.array_equal(B.reps(2 + b), np.array(oreps, dtype=np.uint64)), lab


@pytest.mark.parametrize("n,stride,refl", [(16, 1, True), (17, 1, True), (18, 1, False), (18, 2, True),
                                           (20, 1, True), (20, 4, True)])
def test_orbits_bit_exact_large(lib, n, stride, refl):
    """Orbit lists up to 20 qubits (2^20 states) bit for bit against the brute-force
    oracle over explicit permutations; block sizes against the character formula."""
    print(f"orbits n={n} stride={stride} refl={refl}", flush=True)
    B = lib.Basis(n, _group(refl), stride)
    reps, _ = obasis.orbit_reps(n, stride, refl)
    assert np.array_equal(B.reps(0), reps.astype(np.uint64))
    if refl:
        creps, _ = obasis.orbit_reps(n, stride, False)
        assert np.array_equal(B.reps(1), creps.astype(np.uint64))
    sizes = counts.block_sizes(n, stride, refl)
    labs = [l for l in counts.irrep_labels(n // stride, refl) if sizes[l][0] > 0]
    assert B.sizes == [sizes[l][0] for l in labs]
    assert B.dim == 2 ** n


@pytest.mark.parametrize("n", [16, 20, 22, 24, 26, 28, 30])
def test_orbit_counts_large(lib, n):
    """Orbit counts up to the library's limit of 30 qubits (2^30 states canonicalised on the
    device) against Burnside's necklace and bracelet counts (Table I's D_n column)."""
    print(f"orbit counts n={n}", flush=True)
    B = lib.Basis(n, "dihedral", 1)
    assert len(B.reps(0)) == counts.bracelets(n)
    assert len(B.reps(1)) == counts.necklaces(n)
    assert B.sizes[0] == counts.bracelets(n)
    assert B.dim == 2 ** n
    del B


@pytest.mark.parametrize("n,stride,refl", [(4, 1, True), (6, 1, True), (7, 1, True), (8, 2, True), (6, 1, False),
                                           (9, 3, True)])
def test_state_maps_match_oracle_basis(lib, n, stride, refl):
    import torch
    print(f"state maps n={n} stride={stride} refl={refl}", flush=True)
    B = lib.Basis(n, _group(refl), stride)
    rng = np.random.default_rng(n * 10 + stride)
    psi = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    expect = []
    for lab in counts.irrep_labels(n // stride, refl):
        Vs, _ = obasis.convention_basis(n, lab, stride, refl)
        if Vs[0].shape[1] == 0:
            continue
        for V in Vs:
            expect.append(V.conj().T @ psi)
    expect = np.concatenate(expect)
    got = B.to_blocks(torch.tensor(psi, device="cuda")).cpu().numpy()
    assert np.abs(got - expect).max() < 1e-12
    back = B.from_blocks(torch.tensor(expect, device="cuda")).cpu().numpy()
    assert np.abs(back - psi).max() < 1e-12
