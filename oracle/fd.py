"""Slice-local central finite differences of the objective (FP64).

Changing u[j, k] alters only U_j, so o(u + h e_jk) = <lambda_{j+1}| U_j(u_j + h e_k) |psi_j>
exactly; each probe costs one propagator, not a sweep.  The norm ||psi_N|| does not
depend on u (unitarity), so the FD quotient of |o|^2 is divided by the same norms as F.
"""
from __future__ import annotations

import numpy as np

from . import grape


def fd_gradient(blocks, u, dt, psi0, psif, entries, h=1e-4):
    u = np.asarray(u, float)
    N = u.shape[0]
    fw, bw = grape.sweeps(blocks, u, dt, psi0, psif)
    nN = sum(float(np.sum(np.abs(fw[b][N]) ** 2)) for b in range(len(blocks)))
    nf = sum(float(np.sum(np.abs(psif[b]) ** 2)) for b in range(len(blocks)))
    out = []
    for (j, k) in entries:
        vals = []
        for sgn in (+1.0, -1.0):
            uj = u[j].copy()
            uj[k] += sgn * h
            o = 0.0
            for b, blk in enumerate(blocks):
                U = grape.propagator(blk["H0"], blk["Hk"], uj, dt)
                o = o + np.sum(np.conj(bw[b][j + 1]) * (U @ fw[b][j]))
            vals.append(abs(o) ** 2)
        out.append((vals[0] - vals[1]) / (2 * h) / (nN * nf))
    return np.array(out)
