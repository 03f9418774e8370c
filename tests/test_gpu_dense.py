"""The block-reduced hot path against the same hot path on the dense 2^n space (the
trivial group: rotation by n sites, no reflection, one block of 2^n states).  The
symmetry transformation is unitary, so the objective and every gradient entry agree
(Sec. II A: the reduced problem reaches the same result)."""
import numpy as np
import pytest

import qoc_workloads as W
from oracle import grape as og
from tests._common import FP32_GRAD_REL, oracle_blocks, panels_from_flat

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tf,tg", [("c128", 1e-12, 1e-12), ("c64", 1e-6, FP32_GRAD_REL)])
def test_dense_equals_blocks(lib, prec, tf, tg):
    import torch
    n, N, dt = 10, 8, 0.02
    print(f"dense vs blocks {prec} n={n} N={N}", flush=True)
    rng = np.random.default_rng(21)
    h0 = W.heisenberg_ring_terms(0.9)
    hk = W.global_controls()
    u = torch.tensor(rng.uniform(-2, 2, (N, 2)), device="cuda")
    B = lib.Basis(n)
    S = lib.System(B, h0, hk)
    P = lib.Plan(S, prec, N, dt, 2.0)
    p0 = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    pf = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    ob, gb = lib.fidelity_grad(P, u, p0, pf)
    Bd = lib.Basis(n, "cyclic", n)
    assert Bd.sizes == [2 ** n]
    d0, df = B.from_blocks(p0), B.from_blocks(pf)
    assert torch.equal(Bd.to_blocks(d0), d0)  # the dense block is the computational basis
    Sd = lib.System(Bd, h0, hk)
    Pd = lib.Plan(Sd, prec, N, dt, 2.0)
    od, gd = lib.fidelity_grad(Pd, u, d0, df)
    dF = abs(od[0].item() - ob[0].item())
    dg = (gd - gb).abs().max().item()
    print(f"  F {ob[0].item():.12f}  |dF| {dF:.2e}  max|dg| {dg:.2e}", flush=True)
    assert dF <= tf
    assert dg <= tg * (gb.abs().max().item() if prec == "c64" else 1.0) + (1e-9 if prec == "c64" else 0.0)
    # both against the oracle's block route
    blocks = oracle_blocks(n, h0, hk)
    ref = og.fidelity_grad(blocks, u.cpu().numpy(), dt, panels_from_flat(blocks, p0.cpu().numpy()),
                           panels_from_flat(blocks, pf.cpu().numpy()))
    gmax = np.abs(ref["grad"]).max()
    for o, g in ((ob, gb), (od, gd)):
        assert abs(o[0].item() - ref["F"]) <= tf
        assert np.abs(g.cpu().numpy() - ref["grad"]).max() <= (tg * gmax + 1e-9 if prec == "c64" else tg)
