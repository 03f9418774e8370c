"""Pins for the oracle's gate propagation and gate fidelity (oracle/gate.py): the block
route against the dense 2^n route, a single slice against scipy's expm, the separable
ring against Kronecker products of 2 x 2 rotations, and the fidelity's invariances."""
import numpy as np
import pytest
from scipy.linalg import expm

import qoc_workloads as W
from oracle import gate, grape, pauli


def _controls(seed, N, K=2, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, (N, K))


@pytest.mark.parametrize("n", [5, 6])
def test_block_route_equals_dense_route(n):
    """Block-diagonalising the dense K gives the block K's, and the weighted block traces
    give the dense trace (the E blocks count twice)."""
    N, dt = 7, 0.1
    h0 = W.full_coupling_terms(n, 1.0, [0.7, 0.3, 0.2][: n // 2]) + [W.ring_pair(0.4, "xx")]
    hk = W.global_controls(0.5)
    dense = grape.dense_system(n, h0, hk)
    blocks = grape.block_system(n, h0, hk)
    ua, ub = _controls(1, N), _controls(2, N)
    Kda, Kdb = gate.gate_unitaries(dense, ua, dt)[0], gate.gate_unitaries(dense, ub, dt)[0]
    Ka, Kb = gate.gate_unitaries(blocks, ua, dt), gate.gate_unitaries(blocks, ub, dt)
    for b, K in zip(blocks, Ka):
        for V in b["V"]:
            assert np.abs(V.conj().T @ Kda @ V - K).max() <= 1e-12
    assert sum(b["d"] * b["m"] for b in blocks) == 2 ** n
    fd = gate.gate_fidelity([Kda], [Kdb], [1])
    fb = gate.gate_fidelity(Ka, Kb, [b["d"] for b in blocks])
    assert abs(fd["t"] - np.trace(Kda.conj().T @ Kdb)) <= 1e-12 * 2 ** n
    assert abs(fb["t"] - fd["t"]) <= 1e-11 * 2 ** n
    assert abs(fb["F"] - fd["F"]) <= 1e-12 and fb["D"] == 2 ** n
    # unitaries: the norm-normalised F is the paper's |Tr / 2^n|^2
    assert abs(fb["na"] - 2 ** n) <= 1e-10 and abs(fb["F"] - fb["F_paper"]) <= 1e-12


def test_single_slice_is_the_matrix_exponential():
    n, dt = 4, 0.3
    h0, hk = W.ising_ring_terms(1.0, 0.6), W.global_controls(0.5)
    dense = grape.dense_system(n, h0, hk)
    u = _controls(3, 1)
    H = pauli.hamiltonian(n, h0).toarray() + sum(u[0, k] * pauli.hamiltonian(n, t).toarray()
                                                  for k, t in enumerate(hk))
    K = gate.gate_unitaries(dense, u, dt)[0]
    assert np.abs(K - expm(-1j * dt * H)).max() <= 1e-13


def test_separable_ring_is_a_product_of_single_qubit_rotations():
    """Without coupling every qubit evolves alone under (B_z/2) sigma_z + (u_x sigma_x +
    u_y sigma_y)/2, so K = k (x) k (x) ... (x) k with k the 2 x 2 time-ordered product."""
    n, N, dt = 3, 9, 0.2
    h0, hk = [W.one_body(0.5, "z")], W.global_controls(0.5)
    u = _controls(4, N)
    sx = np.array([[0, 1], [1, 0]], complex)
    sy = np.array([[0, -1j], [1j, 0]])
    sz = np.diag([1.0 + 0j, -1.0])
    k = np.eye(2, dtype=complex)
    for j in range(N):
        k = expm(-1j * dt * (0.5 * sz + 0.5 * u[j, 0] * sx + 0.5 * u[j, 1] * sy)) @ k
    ref = k
    for _ in range(n - 1):
        ref = np.kron(ref, k)
    K = gate.gate_unitaries(grape.dense_system(n, h0, hk), u, dt)[0]
    assert np.abs(K - ref).max() <= 1e-12


def test_fidelity_invariances():
    n, N, dt = 5, 6, 0.1
    blocks = grape.block_system(n, W.ising_ring_terms(1.0, 1.0), W.global_controls(0.5))
    w = [b["d"] for b in blocks]
    Ka = gate.gate_unitaries(blocks, _controls(5, N), dt)
    Kb = gate.gate_unitaries(blocks, _controls(6, N), dt)
    assert abs(gate.gate_fidelity(Ka, Ka, w)["F"] - 1.0) <= 1e-13
    phase = np.exp(0.7j)
    f1 = gate.gate_fidelity(Ka, Kb, w)["F"]
    f2 = gate.gate_fidelity(Ka, [phase * K for K in Kb], w)["F"]
    assert abs(f1 - f2) <= 1e-14 and 0.0 <= f1 < 1.0
    # a non-unitary scale drops out of F but not out of F_paper
    f3 = gate.gate_fidelity(Ka, [1.01 * K for K in Ka], w)
    assert abs(f3["F"] - 1.0) <= 1e-13 and abs(f3["F_paper"] - 1.01 ** 2) <= 1e-12
    for K in Ka:
        assert np.abs(K.conj().T @ K - np.eye(K.shape[0])).max() <= 1e-12
