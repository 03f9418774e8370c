"""The hot path captured into a HIP graph: every replay equals the eager call, with the
program's own eager work and synchronisations between replays; new controls copied into
the captured input change the result exactly as an eager call would."""
import numpy as np
import pytest

import qoc_workloads as W
from tests._common import all_states, flat_from_panels, oracle_blocks

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_graph_replays_match_eager(lib, prec):
    import torch
    print(f"graph capture {prec}", flush=True)
    w = W.config1(N=60)
    ob = oracle_blocks(6, w.h0, w.hk)
    psi0, psif = all_states(ob, np.random.default_rng(3))
    B = lib.Basis(6)
    S = lib.System(B, w.h0, w.hk)
    P = lib.Plan(S, prec, w.N, w.dt, 1.0)
    u = torch.tensor(w.u, device="cuda")
    p0 = torch.tensor(flat_from_panels(psi0), device="cuda")
    pf = torch.tensor(flat_from_panels(psif), device="cuda")
    o_e, g_e = lib.fidelity_grad(P, u, p0, pf)
    o_e, g_e = o_e.clone(), g_e.clone()
    step = lib.CapturedStep(P, u, p0, pf)
    for rep in range(4):
        out, grad = step.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, o_e) and torch.equal(grad, g_e), rep
        # unrelated eager work and a second eager call between replays
        _ = (torch.randn(256, 256, device="cuda") @ torch.randn(256, 256, device="cuda")).sum().item()
        o2, g2 = lib.fidelity_grad(P, u, p0, pf, workspace=torch.empty(P.workspace_bytes, dtype=torch.uint8,
                                                                        device="cuda"))
        assert torch.equal(o2, o_e)
    # new controls through the captured input tensor
    u_new = torch.tensor(np.random.default_rng(9).uniform(-1, 1, (w.N, 2)), device="cuda")
    o_n, g_n = lib.fidelity_grad(P, u_new, p0, pf, workspace=torch.empty(P.workspace_bytes, dtype=torch.uint8,
                                                                          device="cuda"))
    step.u.copy_(u_new)
    out, grad = step.replay()
    torch.cuda.synchronize()
    assert torch.equal(out, o_n) and torch.equal(grad, g_n)
