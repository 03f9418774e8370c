"""Pins for the oracle's Trotterised per-qubit-control propagator (oracle/lts.py, Sec. III B,
Eqs. (8)-(11)): the swap / repeated-block form of Eq. (11) against the direct form of
Eq. (10), exactness without coupling, first-order Trotter error, the qubit-by-qubit state
route against the dense one, and unitarity."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import gate, lts, pauli


def _u(seed, N, n):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (N, 2 * n))


@pytest.mark.parametrize("n", [3, 4, 5])
def test_transformed_form_equals_direct_form(n):
    uj = _u(n, 1, n)[0]
    D = lts.slice_direct(n, 1.0, 0.8, uj, 0.05)
    T = lts.slice_transformed(n, 1.0, 0.8, uj, 0.05)
    assert np.abs(D - T).max() <= 1e-12


def test_swap_moves_a_qubit_operator_to_the_last_qubit():
    n = 4
    for i in range(1, n + 1):
        A = lts.swap_matrix(n, i, n)
        for a in "xyz":
            lhs = A.T @ pauli.pauli_string(n, {i: a}).toarray() @ A
            assert np.abs(lhs - pauli.pauli_string(n, {n: a}).toarray()).max() == 0.0


def test_no_coupling_is_exact():
    """With c_cpl = 0 the qubit factors act on different qubits and commute, so the split
    has no error: U^LTS = exp(-i tau H_j)."""
    n, dt = 4, 0.3
    uj = _u(7, 1, n)[0]
    assert np.abs(lts.slice_direct(n, 1.0, 0.0, uj, dt) - lts.exact_slice(n, 1.0, 0.0, uj, dt)).max() <= 1e-13


def test_trotter_error_is_second_order_per_step():
    """One step of a first-order splitting errs by O(tau^2): halving tau quarters it."""
    n = 4
    uj = _u(8, 1, n)[0]
    errs = []
    for dt in (0.08, 0.04, 0.02):
        errs.append(np.abs(lts.slice_direct(n, 1.0, 1.0, uj, dt) - lts.exact_slice(n, 1.0, 1.0, uj, dt)).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.2 < r1 < 4.8 and 3.2 < r2 < 4.8


def test_state_route_equals_dense_route_and_is_unitary():
    n, N, dt = 4, 5, 0.1
    u = _u(9, N, n)
    K = lts.lts_gate(n, 1.0, 0.7, u, dt)
    assert np.abs(lts.apply_state(n, 1.0, 0.7, u, dt, np.eye(2 ** n)) - K).max() <= 1e-12
    assert np.abs(K.conj().T @ K - np.eye(2 ** n)).max() <= 1e-12
    # the coupling factor is diagonal: exp of the dense coupling is diagonal too
    C = expm(-1j * 0.1 * lts.coupling(n, 0.7))
    assert np.abs(C - np.diag(np.diag(C))).max() == 0.0


def test_lts_gate_fidelity_close_to_exact_for_small_steps():
    """The gate fidelity of K^LTS against the exact K (Sec. III B's comparison) approaches 1
    as tau shrinks, with the error falling as tau^2 for a fixed total time."""
    n, T = 4, 1.0
    base = _u(10, 8, n)
    fs = []
    for N in (8, 16):
        u = np.repeat(base, N // 8, axis=0)
        dt = T / N
        fs.append(1.0 - gate.gate_fidelity([lts.lts_gate(n, 1.0, 1.0, u, dt)], [lts.exact_gate(n, 1.0, 1.0, u, dt)],
                                           [1])["F"])
    assert 0.0 < fs[1] < fs[0] < 1e-2
    assert 2.5 < fs[0] / fs[1] < 6.0


def _states(seed, n):
    rng = np.random.default_rng(seed)
    p0 = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    pf = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    return p0 / np.linalg.norm(p0), pf / np.linalg.norm(pf)


def test_trotterised_gradient_matches_central_differences():
    n, N, dt, h = 4, 3, 0.1, 1e-5
    u = _u(60, N, n)
    p0, pf = _states(61, n)
    r = lts.fidelity_grad(n, 1.0, 0.8, u, dt, p0, pf)
    assert abs(r["F"] - abs(np.vdot(pf, lts.lts_gate(n, 1.0, 0.8, u, dt) @ p0)) ** 2) <= 1e-13
    fd = np.zeros_like(u)
    for j in range(N):
        for k in range(2 * n):
            up, um = u.copy(), u.copy()
            up[j, k] += h
            um[j, k] -= h
            fd[j, k] = (lts.fidelity_grad(n, 1.0, 0.8, up, dt, p0, pf)["F"]
                        - lts.fidelity_grad(n, 1.0, 0.8, um, dt, p0, pf)["F"]) / (2 * h)
    assert np.abs(fd - r["grad"]).max() <= 1e-9 * max(1.0, np.abs(r["grad"]).max()) + 1e-10


def test_without_coupling_the_gradient_is_the_exact_grape_gradient():
    """c_cpl = 0: the split is exact, so objective and gradient equal those of the exact
    propagators (the dense GRAPE oracle with 2n per-qubit control operators)."""
    from oracle import grape
    n, N, dt = 3, 4, 0.1
    u = _u(62, N, n)
    p0, pf = _states(63, n)
    h0 = [{"kind": "one_body", "coeff": 0.5, "op": "z", "sites": "all", "stagger": False}]
    hk = []
    for i in range(1, n + 1):
        for a in "XY":
            s = ["I"] * n
            s[i - 1] = a
            hk.append([{"kind": "pauli", "coeff": 0.5, "string": "".join(s)}])
    ref = grape.fidelity_grad(grape.dense_system(n, h0, hk), u, dt, [p0[:, None]], [pf[:, None]])
    r = lts.fidelity_grad(n, 1.0, 0.0, u, dt, p0, pf)
    assert abs(r["F"] - ref["F"]) <= 1e-13
    assert np.abs(r["grad"] - np.asarray(ref["grad"])).max() <= 1e-12
