"""Pauli-sum operators on n qubits (Sec. II A).

sigma_a^(i) = I_2^{(x)(i-1)} (x) sigma_a (x) I_2^{(x)(n-i)}: qubit 1 is the
leftmost Kronecker factor, hence the most significant bit of the basis index.
Bit value 0 is spin up (sigma_z = +1).  Matrices are built with explicit
Kronecker products, with no reliance on bit tricks, so that they can serve as
the definition the rest of the code is checked against.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SIGMA = {
    "i": np.eye(2, dtype=complex),
    "x": np.array([[0, 1], [1, 0]], dtype=complex),
    "y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "z": np.array([[1, 0], [0, -1]], dtype=complex),
}


def pauli_string(n: int, ops: dict) -> sp.csr_matrix:
    """Kronecker product over qubits 1..n; ``ops`` maps qubit -> 'x'|'y'|'z'."""
    out = sp.identity(1, dtype=complex, format="csr")
    for q in range(1, n + 1):
        out = sp.kron(out, sp.csr_matrix(SIGMA[ops.get(q, "i")]), format="csr")
    return out


def _selected(n, sites):
    if sites == "all":
        return list(range(1, n + 1))
    if sites == "even":
        return [q for q in range(1, n + 1) if q % 2 == 0]
    if sites == "odd":
        return [q for q in range(1, n + 1) if q % 2 == 1]
    raise ValueError(sites)


def term_matrix(n: int, term: dict) -> sp.csr_matrix:
    """Sparse matrix of one term descriptor (see qoc_workloads)."""
    kind = term["kind"]
    c = term["coeff"]
    acc = sp.csr_matrix((2 ** n, 2 ** n), dtype=complex)
    if kind == "one_body":
        for q in _selected(n, term["sites"]):
            w = (-1.0) ** q if term.get("stagger") else 1.0
            acc = acc + w * pauli_string(n, {q: term["op"]})
    elif kind == "ring_pair":
        a, b = term["op"][0], term["op"][1]
        d = term["distance"]
        for q in range(1, n + 1):
            q2 = (q - 1 + d) % n + 1
            if q2 == q:
                raise ValueError("ring pair at distance 0 mod n")
            if a == b:
                # sigma_a^(q) sigma_a^(q2): both factors commute, any order.
                acc = acc + pauli_string(n, {q: a, q2: a})
            else:
                acc = acc + (pauli_string(n, {q: a}) @ pauli_string(n, {q2: b}))
    elif kind == "all_pairs":
        a, b = term["op"][0], term["op"][1]
        for q in range(1, n + 1):
            for q2 in range(q + 1, n + 1):
                acc = acc + (pauli_string(n, {q: a}) @ pauli_string(n, {q2: b}))
    elif kind == "pauli":
        s = term["string"]
        if len(s) != n:
            raise ValueError("Pauli string length must equal n")
        acc = acc + pauli_string(n, {q + 1: ch.lower() for q, ch in enumerate(s) if ch.upper() != "I"})
    else:
        raise ValueError(kind)
    return (c * acc).tocsr()


def hamiltonian(n: int, terms) -> sp.csr_matrix:
    H = sp.csr_matrix((2 ** n, 2 ** n), dtype=complex)
    for t in terms:
        H = H + term_matrix(n, t)
    return H.tocsr()
