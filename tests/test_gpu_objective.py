"""Objective-only evaluation, the sweeps' states, autograd and numeric-failure reporting.

* qoc_fidelity (propagators + forward sweep + overlap, Eqs. (3)-(4)) gives the same
  objective as qoc_fidelity_grad bit for bit, on one-segment, segmented and batched plans.
* The states read back satisfy the sweep invariants: o = <lambda_j|psi_j> for every j, and
  the slice-local identity o(u + h e_jk) = <lambda_{j+1}| U_j(u_j + h e_k) |psi_j> gives
  central differences of F that match the gradient (App. B).
* torch.autograd.gradcheck of GrapeFidelity in FP64, and the objective-only path of
  GrapeFidelity.apply when no gradient can be asked for.
* Non-finite controls or states set status bit 1 and raise QocError(QOC_ERR_NUMERIC).
"""
import numpy as np
import pytest

import qoc_workloads as W
from oracle import grape as og
from tests._common import all_states, flat_from_panels, oracle_blocks, plan_with_segments

pytestmark = pytest.mark.gpu


def _ring(lib, n, N, seed, prec="c128", max_ws=0):
    import torch
    w = W.config2(seed=seed, N=N, n=n, variant="all")
    ob = oracle_blocks(n, w.h0, w.hk)
    psi0, psif = all_states(ob, np.random.default_rng(seed + 100))
    B = lib.Basis(n)
    S = lib.System(B, w.h0, w.hk)
    P = lib.Plan(S, prec, N, w.dt, 2.0, max_ws)
    dev = (torch.tensor(w.u, device="cuda"), torch.tensor(flat_from_panels(psi0), device="cuda"),
           torch.tensor(flat_from_panels(psif), device="cuda"))
    return w, ob, psi0, psif, B, S, P, dev


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_objective_only_equals_full_call(lib, prec):
    import torch
    print(f"objective only {prec}", flush=True)
    w, ob, psi0, psif, B, S, P, (u, p0, pf) = _ring(lib, 10, 120, 1, prec)
    out_full, _ = lib.fidelity_grad(P, u, p0, pf)
    out_obj = lib.fidelity(P, u, p0, pf)
    assert torch.equal(out_full[:6], out_obj[:6]) and out_obj[7].item() == 0
    # a segmented plan: the forward pass forms each segment once
    Ps = plan_with_segments(lib, S, prec, w.N, w.dt, 2.0)
    out_seg = lib.fidelity(Ps, u, p0, pf)
    assert torch.equal(out_seg[:6], out_full[:6])
    if prec == "c128":
        ref = og.fidelity_grad(ob, w.u, w.dt, psi0, psif)
        assert abs(out_obj[0].item() - ref["F"]) <= 1e-12


def test_objective_only_batched(lib):
    import torch
    print("objective only batched", flush=True)
    rng = np.random.default_rng(31)
    ws, states = [], []
    for n, N in ((6, 17), (8, 40), (4, 9)):
        u = rng.uniform(-1, 1, (N, 2))
        ws.append(W.Workload(f"ring{n}", n, "dihedral", 1, W.heisenberg_ring_terms(0.8), W.global_controls(), N,
                             0.05, u))
        states.append((W.gaussian_panel(rng, 2 ** n), W.gaussian_panel(rng, 2 ** n)))
    systems = [lib.System(lib.Basis(w.n), w.h0, w.hk) for w in ws]
    P = lib.Plan.batched(systems, "c128", [w.N for w in ws], [w.dt for w in ws], 1.0)
    us = [torch.tensor(w.u, device="cuda") for w in ws]
    p0 = [torch.tensor(s[0], device="cuda") for s in states]
    pf = [torch.tensor(s[1], device="cuda") for s in states]
    out_full, _ = lib.fidelity_grad_batched(P, us, p0, pf)
    out_obj = lib.fidelity_batched(P, us, p0, pf)
    assert torch.equal(out_full[:, :6], out_obj[:, :6])


@pytest.mark.parametrize("prec,segmented", [("c128", False), ("c128", True), ("c64", False)])
def test_state_invariants_and_slice_local_differences(lib, prec, segmented):
    """o = <lambda_j|psi_j> at every j (to the precision's rounding), psi_0 / lambda_N equal
    the inputs, psi_N and lambda_1 match the oracle's sweeps (FP64), and, FP64 only, central
    differences of F through the slice-local identity match the library's gradient."""
    import torch
    print(f"state invariants {prec} segmented={segmented}", flush=True)
    n, N = 8, 30
    w, ob, psi0, psif, B, S, P, (u, p0, pf) = _ring(lib, n, N, 2, prec)
    if segmented:
        P = plan_with_segments(lib, S, prec, N, w.dt, 2.0)
    out, grad = lib.fidelity_grad(P, u, p0, pf)
    o = complex(out[2].item(), out[3].item())
    tol = 1e-12 if prec == "c128" else 2e-5
    assert torch.allclose(lib.read_state(P, "psi", 0), p0.to(torch.complex128), atol=tol if prec == "c64" else 0)
    assert torch.allclose(lib.read_state(P, "lambda", N), pf.to(torch.complex128), atol=tol if prec == "c64" else 0)
    for j in (1, 7, 15, N):
        lam = lib.read_state(P, "lambda", j).cpu().numpy()
        psi = lib.read_state(P, "psi", j).cpu().numpy()
        assert abs(np.vdot(lam, psi) - o) <= tol * max(1.0, abs(o)), j
    if prec != "c128":
        return
    fw, bw = og.sweeps(ob, w.u, w.dt, psi0, psif)
    assert np.abs(lib.read_state(P, "psi", N).cpu().numpy() - flat_from_panels([f[N] for f in fw])).max() <= 1e-12
    assert np.abs(lib.read_state(P, "lambda", 1).cpu().numpy() - flat_from_panels([b[1] for b in bw])).max() <= 1e-12
    # slice-local central differences with the library's own one-slice plan
    h = 1e-4
    P1 = lib.Plan(S, "c128", 1, w.dt, 2.0 + 2 * h)
    norms = out[4].item() * out[5].item()
    g = grad.cpu().numpy()
    for (j, k) in ((0, 0), (4, 1), (17, 0), (N - 1, 1)):
        psi_j = lib.read_state(P, "psi", j)
        lam_j1 = lib.read_state(P, "lambda", j + 1)
        vals = []
        for sgn in (1.0, -1.0):
            uj = u[j:j + 1].clone()
            uj[0, k] += sgn * h
            o1 = lib.fidelity(P1, uj, psi_j, lam_j1)
            vals.append(o1[1].item())
        fd = (vals[0] - vals[1]) / (2 * h) / norms
        assert abs(fd - g[j, k]) <= 1e-9 + 1e-6 * abs(g[j, k]), (j, k, fd, g[j, k])


def test_gradcheck_fp64(lib):
    """torch.autograd.gradcheck of GrapeFidelity (complex128 plan, n = 6, 8 slices)."""
    import torch
    print("gradcheck", flush=True)
    w = W.config1(N=8)
    ob = oracle_blocks(6, w.h0, w.hk)
    psi0, psif = all_states(ob, np.random.default_rng(3))
    B = lib.Basis(6)
    S = lib.System(B, w.h0, w.hk)
    P = lib.Plan(S, "c128", 8, w.dt, 2.0)
    p0 = torch.tensor(flat_from_panels(psi0), device="cuda")
    pf = torch.tensor(flat_from_panels(psif), device="cuda")
    u = torch.tensor(w.u, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: lib.GrapeFidelity.apply(x, P, p0, pf), (u,), eps=1e-6, atol=1e-8,
                                    rtol=1e-6)
    # no gradient requested: the objective alone, same value
    with torch.no_grad():
        F0 = lib.GrapeFidelity.apply(u, P, p0, pf)
    F1 = lib.GrapeFidelity.apply(u, P, p0, pf)
    assert not F0.requires_grad and F1.requires_grad
    assert F0.item() == F1.item()


@pytest.mark.parametrize("where", ["control", "psi0", "psif"])
def test_non_finite_input_is_reported(lib, where):
    import torch
    print(f"non-finite {where}", flush=True)
    w, ob, psi0, psif, B, S, P, (u, p0, pf) = _ring(lib, 6, 20, 4)
    if where == "control":
        u = u.clone()
        u[3, 1] = float("nan")
    elif where == "psi0":
        p0 = p0.clone()
        p0[5] = complex(float("inf"), 0.0)
    else:
        pf = pf.clone()
        pf[2] = complex(0.0, float("nan"))
    out, _ = lib.fidelity_grad(P, u, p0, pf, check=False)
    assert int(out[7].item()) & 2
    with pytest.raises(lib.QocError) as e:
        lib.check_flags(out)
    assert e.value.status == 6 and "non-finite" in str(e.value)
    with pytest.raises(lib.QocError):
        lib.fidelity(P, u, p0, pf)
