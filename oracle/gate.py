"""Gate propagation and gate fidelity, FP64 (test infrastructure only).

The unitary a pulse implements is the time-ordered product of the slice propagators of
Eq. (3), K = U_{N-1} ... U_1 U_0.  Sec. III B compares two such unitaries K_a, K_b of an
n-qubit system by F = |Tr(K_a^dag K_b) / 2^n|^2.  In the symmetry-adapted basis both are
block diagonal, every block theta repeated d_theta times (the dimension of its irrep,
App. A), so Tr(K_a^dag K_b) = sum_theta d_theta Tr(K_a,theta^dag K_b,theta) and
2^n = sum_theta d_theta m_theta.  Over a subset of the blocks the same sums give the
fidelity restricted to their subspace.
"""
from __future__ import annotations

import numpy as np

from . import grape


def gate_unitaries(blocks, u, dt):
    """K = U_{N-1} ... U_0 for every block (list of m x m complex128), slice by slice."""
    u = np.asarray(u, dtype=float)
    out = []
    for b in blocks:
        K = np.eye(b["H0"].shape[0], dtype=complex)
        for j in range(u.shape[0]):
            K = grape.propagator(b["H0"], b["Hk"], u[j], dt) @ K
        out.append(K)
    return out


def gate_fidelity(Ka, Kb, weights):
    """t = sum_theta w_theta Tr(Ka_theta^dag Kb_theta), D = sum_theta w_theta m_theta,
    F_paper = |t|^2 / D^2 and F = |t|^2 / (na nb) with na = sum_theta w_theta ||Ka_theta||_F^2
    (nb likewise), which equals F_paper for unitaries and is what the library reports."""
    t = sum(w * np.trace(a.conj().T @ b) for a, b, w in zip(Ka, Kb, weights))
    D = float(sum(w * a.shape[0] for a, w in zip(Ka, weights)))
    na = float(sum(w * np.sum(np.abs(a) ** 2) for a, w in zip(Ka, weights)))
    nb = float(sum(w * np.sum(np.abs(b) ** 2) for b, w in zip(Kb, weights)))
    return {"F": abs(t) ** 2 / (na * nb), "F_paper": abs(t) ** 2 / D ** 2, "t": t, "D": D, "na": na, "nb": nb}
