"""SU(2) product-state closed form for isotropic Heisenberg rings (test pin).

For H0 = hz sum sigma_z + J sum_i sigma^(i).sigma^(i+1) and global controls
u_k s_k sum sigma_{a_k}, the isotropic coupling commutes with the total spin,
hence with every other term, so
    U_{N-1} ... U_0 = exp(-i T J H_heis) (r_{N-1} ... r_0)^{(x) n},
    r_j = exp(-i dt (hz sigma_z + sum_k u[j,k] s_k sigma_{a_k}))  (2 x 2).
From the all-up state the product state v^{(x)n}, v = r_{N-1}...r_0 |up>, lies in
the symmetric subspace where every bond sigma.sigma equals +1, so the coupling
contributes the phase exp(-i T J n).  The gradient follows by the product rule
through the 2 x 2 chain, with the exact 2 x 2 Frechet derivative of exp.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm, expm_frechet

S = {"x": np.array([[0, 1], [1, 0]], complex), "y": np.array([[0, -1j], [1j, 0]]),
     "z": np.array([[1, 0], [0, -1]], complex)}


def _qubit_table(n):
    x = np.arange(2 ** n)
    # bit of qubit q (1-based) is bit position n - q
    return [((x >> (n - q)) & 1) for q in range(1, n + 1)]


def fidelity_grad(n, hz, J, controls, u, dt, psif_dense):
    """controls: list of (axis, scale); u (N, K); psif_dense on the full 2^n space."""
    u = np.asarray(u, float)
    N, K = u.shape
    gens = [(-1j * dt) * sc * S[a] for a, sc in controls]
    base = (-1j * dt) * hz * S["z"]
    r = [expm(base + sum(u[j, k] * gens[k] for k in range(K))) for j in range(N)]
    # prefix (right) and suffix (left) products
    pre = [np.eye(2, dtype=complex)]
    for j in range(N):
        pre.append(r[j] @ pre[-1])
    suf = [np.eye(2, dtype=complex)] * (N + 1)
    for j in range(N - 1, -1, -1):
        suf[j] = suf[j + 1] @ r[j]
    up = np.array([1.0, 0.0], complex)
    v = pre[N] @ up
    bits = _qubit_table(n)
    phase = np.exp(-1j * dt * N * J * n)
    cf = np.conj(psif_dense)
    amps = [v[b] for b in bits]
    prod = np.ones(2 ** n, complex)
    for a in amps:
        prod = prod * a
    o = phase * np.sum(cf * prod)
    # T_vec[c] = sum_q sum_{x: x_q = c} conj(psif[x]) prod_{q' != q} v[x_q']
    Tvec = np.zeros(2, complex)
    for q in range(n):
        others = np.ones(2 ** n, complex)
        for q2 in range(n):
            if q2 != q:
                others = others * amps[q2]
        for c in (0, 1):
            Tvec[c] += np.sum(cf * others * (bits[q] == c))
    g = np.zeros((N, K), complex)
    for j in range(N):
        X = base + sum(u[j, k] * gens[k] for k in range(K))
        for k in range(K):
            dr = expm_frechet(X, gens[k], compute_expm=False)
            dv = suf[j + 1] @ dr @ pre[j] @ up
            g[j, k] = phase * (Tvec @ dv)
    nN = float(np.vdot(v, v).real) ** n
    nf = float(np.vdot(psif_dense, psif_dense).real)
    F = abs(o) ** 2 / (nN * nf)
    grad = 2.0 * np.real(np.conj(o) * g) / (nN * nf)
    return {"F": F, "o": o, "grad": grad}
