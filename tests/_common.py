"""Shared test helpers: oracle systems, panel layout (column-major m x d per block) and
the reader of the stored oracle values under tests/golden/."""
import os

import numpy as np

import qoc_workloads as W
from oracle import grape


def flat_from_panels(panels):
    return np.concatenate([np.asarray(P).flatten(order="F") for P in panels])


def panels_from_flat(blocks, flat):
    out, off = [], 0
    for b in blocks:
        s = b["m"] * b["d"]
        out.append(np.asarray(flat[off:off + s]).reshape(b["d"], b["m"]).T)
        off += s
    return out


def plain_states(blocks, rng):
    """psi0 = first basis state of the first block (all-up), psi_f Gaussian in the first block."""
    m0 = blocks[0]["m"]
    pf = W.gaussian_panel(rng, m0)
    psif = [pf[:, None]] + [np.zeros((b["m"], b["d"]), complex) for b in blocks[1:]]
    psi0 = [np.eye(m0, dtype=complex)[:, [0]]] + [np.zeros((b["m"], b["d"]), complex) for b in blocks[1:]]
    return psi0, psif


def all_states(blocks, rng):
    """psi_f then psi0: independent normalised Gaussians over every block and copy."""
    D = sum(b["m"] * b["d"] for b in blocks)
    vf = W.gaussian_panel(rng, D)
    v0 = W.gaussian_panel(rng, D)
    return panels_from_flat(blocks, v0), panels_from_flat(blocks, vf)


def oracle_blocks(n, h0, hk, group="dihedral", stride=1):
    return grape.block_system(n, h0, hk, group, stride, "convention")


# FP32 (complex64) gradient bound relative to max|g|.  Each complex64 propagator carries a
# relative rounding error of about u32 sqrt(m) per product (u32 = 6e-8) over ~4 products;
# the states accumulate it over N slices like a random walk, sqrt(N) * 4e-7 ~ 1e-5 at
# N = 1000 in the worst block, and the gradient inherits it relative to its own size.
# Measured on the 12-qubit ring (1000 slices, blocks up to 346): 4.1e-6 max|g|; on the
# 500-slice S_128 candidates and the ragged ring batch: 3e-6 to 1.4e-5.  A start in one
# basis state (the all-up "plain" transfers) has a gradient that is small against the
# rounding scale 2 |o| dt ||H_k|| u32 sqrt(N) of the costates: 2.6e-5 max|g| measured on the
# 12-qubit ring's first block, so those tests pass a bound of their own (5e-5).
FP32_GRAD_REL = 2e-5


def fp32_grad_tol(gmax, rel=FP32_GRAD_REL):
    return rel * gmax + 1e-9


def plan_with_segments(lib, S, prec, N, dt, u_bound, min_segments=2, budget_frac=0.3):
    """A plan whose workspace budget forces at least min_segments segments (propagators
    of earlier segments recomputed in the backward sweep)."""
    full = lib.Plan(S, prec, N, dt, u_bound).workspace_bytes
    frac = budget_frac
    while True:
        P = lib.Plan(S, prec, N, dt, u_bound, int(full * frac))
        if P.info["segments"] >= min_segments:
            return P
        frac *= 0.7
        assert frac > 1e-4


GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _num(tok):
    # values are written as Python float reprs (older files: numpy scalar reprs)
    return float(tok.replace("np.float64(", "").rstrip(")"))


def read_golden(name):
    """(scalars, gradient[N, K]) from a file written by tests/golden/make_golden.py."""
    vals, grad = {}, []
    for line in open(os.path.join(GOLDEN_DIR, name)):
        if line.startswith("#"):
            continue
        k, *v = line.split()
        if k == "g":
            grad.append([_num(x) for x in v])
        else:
            vals[k] = _num(v[0])
    return vals, np.array(grad)
