"""Trotterised propagator for per-qubit controls, FP64 (test infrastructure only).

Sec. III B gives every qubit its own pulse (Eq. (8)) on the Ising ring:
    H_j = sum_i [ (B_z/2) sigma_z^(i) + (1/2)(Bx_i[j] sigma_x^(i) + By_i[j] sigma_y^(i)) ]
          + (c_cpl/4) sum_i sigma_z^(i) sigma_z^(i+1)                                   (Eq. (9))
and splits the slice propagator by symmetry (Eq. (10)):
    U_j^LTS = prod_{i=1..n} [ exp(-i tau (H_0^(i) + H_c'^(i)[j])) exp(-i (tau/n) H_cpl) ]
with H_0^(i) = (B_z/2) sigma_z^(i), H_c'^(i) the qubit's control term and H_cpl the
coupling sum; the product runs i = 1 on the left to i = n on the right, so the factor of
qubit n acts on a state first, and within a bracket the coupling factor acts first.
Eq. (11) writes each bracket through the swap A_i = A_(i,n) of qubits i and n, under
which the qubit-i factor becomes 2^(n-1) identical 2 x 2 blocks on the last qubit, and
the coupling factor through the D_n block diagonalisation A_D.

Controls: u[j, 2(i-1)] = Bx_i[j], u[j, 2(i-1)+1] = By_i[j] (i = 1..n).

Routes: ``slice_direct`` (Eq. (10) with dense exponentials), ``slice_transformed``
(Eq. (11): swaps, repeated 2 x 2 blocks, D_n blocks), ``apply_state`` (the factors of
Eq. (10) applied one qubit at a time to state columns, for sizes where dense matrices do
not fit), ``exact_slice`` (Eq. (3) of the untrotterised H_j).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm, expm_frechet

from . import basis, counts, pauli

SX, SY, SZ = pauli.SIGMA["x"], pauli.SIGMA["y"], pauli.SIGMA["z"]


def qubit_terms(n, Bz, uj, i):
    """H_0^(i) + H_c'^(i) as a dense 2^n matrix."""
    return (0.5 * Bz * pauli.pauli_string(n, {i: "z"}) + 0.5 * uj[2 * (i - 1)] * pauli.pauli_string(n, {i: "x"})
            + 0.5 * uj[2 * (i - 1) + 1] * pauli.pauli_string(n, {i: "y"})).toarray()


def coupling(n, c):
    """H_cpl = (c/4) sum_{i=1..n} sigma_z^(i) sigma_z^(i+1), qubit n+1 = qubit 1 (for n = 2
    the pair appears twice, as in the ring sums of Eqs. (5)-(7))."""
    H = sum(pauli.pauli_string(n, {i: "z"}) @ pauli.pauli_string(n, {i % n + 1: "z"}) for i in range(1, n + 1))
    return (0.25 * c * H).toarray()


def full_hamiltonian(n, Bz, c, uj):
    return sum(qubit_terms(n, Bz, uj, i) for i in range(1, n + 1)) + coupling(n, c)


def exact_slice(n, Bz, c, uj, dt):
    return expm(-1j * dt * full_hamiltonian(n, Bz, c, uj))


def slice_direct(n, Bz, c, uj, dt):
    """Eq. (10) with dense matrix exponentials."""
    C = expm(-1j * (dt / n) * coupling(n, c))
    U = np.eye(2 ** n, dtype=complex)
    for i in range(1, n + 1):
        U = U @ expm(-1j * dt * qubit_terms(n, Bz, uj, i)) @ C
    return U


def swap_matrix(n, i, k):
    """Permutation matrix exchanging qubits i and k (both 1-based)."""
    P = np.zeros((2 ** n, 2 ** n))
    pi, pk = n - i, n - k  # bit positions
    for x in range(2 ** n):
        bi, bk = (x >> pi) & 1, (x >> pk) & 1
        y = x & ~((1 << pi) | (1 << pk)) | (bi << pk) | (bk << pi)
        P[y, x] = 1.0
    return P


def slice_transformed(n, Bz, c, uj, dt):
    """Eq. (11): A_i [I_{2^(n-1)} (x) exp(-i tau h_i)] A_i^dag for the qubit factors, and
    the coupling factor assembled from the exponentials of its D_n blocks."""
    Hc = coupling(n, c)
    Ucpl = np.zeros((2 ** n, 2 ** n), complex)
    for lab in counts.irrep_labels(n, True):
        Vs, _ = basis.convention_basis(n, lab, 1, True)
        if Vs[0].shape[1] == 0:
            continue
        E = expm(-1j * (dt / n) * (Vs[0].conj().T @ Hc @ Vs[0]))
        for V in Vs:
            Ucpl = Ucpl + V @ E @ V.conj().T
    U = np.eye(2 ** n, dtype=complex)
    for i in range(1, n + 1):
        h = 0.5 * Bz * SZ + 0.5 * uj[2 * (i - 1)] * SX + 0.5 * uj[2 * (i - 1) + 1] * SY
        blocks = np.kron(np.eye(2 ** (n - 1)), expm(-1j * dt * h))  # 2^(n-1) identical 2 x 2 blocks
        A = swap_matrix(n, i, n)
        U = U @ (A @ blocks @ A.T) @ Ucpl
    return U


def _apply_qubit(psi, n, i, g):
    """Apply the 2 x 2 matrix g to qubit i of every column of psi (2^n x k)."""
    k = psi.shape[1]
    t = psi.reshape(2 ** (i - 1), 2, 2 ** (n - i), k)
    return np.einsum("ab,xbyk->xayk", g, t).reshape(2 ** n, k)


def apply_state(n, Bz, c, u, dt, psi):
    """psi_N = U_{N-1}^LTS ... U_0^LTS psi for state columns psi (2^n x k)."""
    # the coupling is diagonal: its energy on basis state x, with z_q = +1 for spin up
    zs = np.array([[1.0 if ((x >> (n - q)) & 1) == 0 else -1.0 for q in range(1, n + 1)] for x in range(2 ** n)])
    ecpl = 0.25 * c * sum(zs[:, q - 1] * zs[:, q % n] for q in range(1, n + 1))
    phase = np.exp(-1j * (dt / n) * ecpl)[:, None]
    out = np.array(psi, dtype=complex, copy=True)
    for j in range(np.asarray(u).shape[0]):
        uj = u[j]
        for i in range(n, 0, -1):
            out = phase * out
            h = 0.5 * Bz * SZ + 0.5 * uj[2 * (i - 1)] * SX + 0.5 * uj[2 * (i - 1) + 1] * SY
            out = _apply_qubit(out, n, i, expm(-1j * dt * h))
    return out


def lts_gate(n, Bz, c, u, dt):
    """K^LTS = U_{N-1}^LTS ... U_0^LTS (dense)."""
    K = np.eye(2 ** n, dtype=complex)
    for j in range(np.asarray(u).shape[0]):
        K = slice_direct(n, Bz, c, u[j], dt) @ K
    return K


def exact_gate(n, Bz, c, u, dt):
    K = np.eye(2 ** n, dtype=complex)
    for j in range(np.asarray(u).shape[0]):
        K = exact_slice(n, Bz, c, u[j], dt) @ K
    return K


def qubit_factor(Bz, ux, uy, dt):
    """The 2 x 2 factor exp(-i dt h.sigma) of one qubit, h = (ux, uy, Bz) / 2."""
    return expm(-1j * dt * (0.5 * Bz * SZ + 0.5 * ux * SX + 0.5 * uy * SY))


def fidelity_grad(n, Bz, c, u, dt, psi0, psif):
    """State transfer through the Trotterised propagator (Eq. (10)) and its exact gradient.

    o = <psi_f| U_{N-1}^LTS ... U_0^LTS |psi_0>, F = |o|^2 / (||psi_N||^2 ||psi_f||^2) (the
    objective of Eq. (4)).  The control u[j, 2(i-1)+a] enters only qubit i's factor g of
    slice j, so do/du = <lambda| (dg/du on qubit i) |psi> with psi the state just before
    that factor and lambda the costate just after it (psi_f carried back through the
    adjoints of every later factor); dg/du is the Frechet derivative of the 2 x 2
    exponential in the direction -i dt sigma_a / 2 (scipy's expm_frechet).  Returns F, o,
    the norms and the gradient (N, 2n).  States are stored at every factor: small n only."""
    u = np.asarray(u, dtype=float)
    N = u.shape[0]
    zs = np.array([[1.0 if ((x >> (n - q)) & 1) == 0 else -1.0 for q in range(1, n + 1)] for x in range(2 ** n)])
    ecpl = 0.25 * c * sum(zs[:, q - 1] * zs[:, q % n] for q in range(1, n + 1))
    phase = np.exp(-1j * (dt / n) * ecpl)
    # forward: the sequence of factors, and the state before each qubit factor
    ops, before = [], []
    psi = np.array(psi0, dtype=complex).reshape(-1)
    for j in range(N):
        for i in range(n, 0, -1):
            psi = phase * psi
            before.append(psi)
            g = qubit_factor(Bz, u[j, 2 * (i - 1)], u[j, 2 * (i - 1) + 1], dt)
            ops.append((j, i, g))
            psi = _apply_qubit(psi[:, None], n, i, g)[:, 0]
    psif = np.array(psif, dtype=complex).reshape(-1)
    o = np.vdot(psif, psi)
    nN, nf = float(np.vdot(psi, psi).real), float(np.vdot(psif, psif).real)
    grad = np.zeros((N, 2 * n))
    lam = psif.copy()
    for (j, i, g), pb in zip(reversed(ops), reversed(before)):
        # lam is the costate just after factor (j, i)
        h = 0.5 * Bz * SZ + 0.5 * u[j, 2 * (i - 1)] * SX + 0.5 * u[j, 2 * (i - 1) + 1] * SY
        for a, s in enumerate((SX, SY)):
            _, dg = expm_frechet(-1j * dt * h, -1j * dt * 0.5 * s)
            do = np.vdot(lam, _apply_qubit(pb[:, None], n, i, dg)[:, 0])
            grad[j, 2 * (i - 1) + a] = 2.0 * (np.conj(o) * do).real / (nN * nf)
        lam = _apply_qubit(lam[:, None], n, i, g.conj().T)[:, 0]
        lam = np.conj(phase) * lam
    return {"F": abs(o) ** 2 / (nN * nf), "o": o, "nN": nN, "nf": nf, "grad": grad, "psiN": psi}
