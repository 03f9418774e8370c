"""Batched plans (many independent problems sharing every launch) against the oracle:
a prefix of the 256-ring workload (ragged n and N), candidate pulses under S_n (vs stored
oracle values), and a small FP64 batch checked to the FP64 tolerance."""
import numpy as np
import pytest

import qoc_workloads as W
from oracle import counts
from oracle import grape as og
from tests._common import fp32_grad_tol, panels_from_flat, read_golden

pytestmark = pytest.mark.gpu


def _sizes(n):
    bs = counts.block_sizes(n)
    return [(m, d) for lab, (m, d) in bs.items() if m > 0]


def _problem_states(rng, n):
    D = 2 ** n
    vf = W.gaussian_panel(rng, D)
    v0 = W.gaussian_panel(rng, D)
    return v0, vf


def _oracle(w, v0, vf):
    ob = og.block_system(w.n, w.h0, w.hk, "dihedral", w.stride)
    return og.fidelity_grad(ob, w.u, w.dt, panels_from_flat(ob, v0), panels_from_flat(ob, vf))


def test_ring_batch_prefix(lib):
    """Problems 0..8 of the 256-ring workload (n = 14, 12, 12, 10, 10, 8, 8, 8, 8; 424-1745
    slices) in one FP32 plan, every problem against the FP64 oracle: problems 0, 1, 2 and 4
    against values stored by tests/golden/make_golden.py (their oracle runs take minutes to an
    hour), the others against the oracle run here."""
    import torch
    print("ring batch prefix", flush=True)
    ws, rng = W.config3_list(seed=0)
    ws = ws[:9]
    states = [_problem_states(rng, w.n) for w in ws]
    bases = {n: lib.Basis(n) for n in sorted({w.n for w in ws})}
    systems = [lib.System(bases[w.n], w.h0, w.hk) for w in ws]
    P = lib.Plan.batched(systems, "c64", [w.N for w in ws], [w.dt for w in ws], 1.0, max_workspace_bytes=60 << 30)
    print(f"  plan {P.info}", flush=True)
    out, grads = lib.fidelity_grad_batched(P, [torch.tensor(w.u, device="cuda") for w in ws],
                                           [torch.tensor(s[0], device="cuda") for s in states],
                                           [torch.tensor(s[1], device="cuda") for s in states])
    out = out.cpu().numpy()
    for p, w in enumerate(ws):
        g = grads[p].cpu().numpy()
        assert out[p, 7] == 0
        if p in (0, 1, 2, 4):
            vals, gref = read_golden(f"batch256_p{p}_n{w.n}_N{w.N}.txt")
            ref = {"F": vals["F"], "grad": gref}
        else:
            ref = _oracle(w, *states[p])
        dF = abs(out[p, 0] - ref["F"])
        dg = np.abs(g - ref["grad"]).max()
        gmax = np.abs(ref["grad"]).max()
        print(f"  problem {p} n={w.n} N={w.N}: |dF|={dF:.2e} max|dg|={dg:.2e} ({dg / gmax:.2e} of max|g|)",
              flush=True)
        assert dF <= 1e-6
        assert dg <= fp32_grad_tol(gmax)


def test_small_batch_fp64_exact(lib):
    """Three rings of different n and N in one FP64 plan, each to the FP64 tolerance."""
    import torch
    print("small FP64 batch", flush=True)
    rng = np.random.default_rng(17)
    ws = []
    for n, N in ((4, 7), (6, 23), (5, 12)):
        u = rng.uniform(-1, 1, (N, 2))
        ws.append(W.Workload(f"ring{n}", n, "dihedral", 1, W.heisenberg_ring_terms(0.7 + 0.1 * n),
                             W.global_controls(), N, 0.07, u))
    states = [_problem_states(rng, w.n) for w in ws]
    systems = [lib.System(lib.Basis(w.n), w.h0, w.hk) for w in ws]
    P = lib.Plan.batched(systems, "c128", [w.N for w in ws], [w.dt for w in ws], 1.0)
    out, grads = lib.fidelity_grad_batched(P, [torch.tensor(w.u, device="cuda") for w in ws],
                                           [torch.tensor(s[0], device="cuda") for s in states],
                                           [torch.tensor(s[1], device="cuda") for s in states])
    for p, w in enumerate(ws):
        ref = _oracle(w, *states[p])
        assert abs(out[p, 0].item() - ref["F"]) <= 1e-12
        assert np.abs(grads[p].cpu().numpy() - ref["grad"]).max() <= 1e-12


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_symmetric_candidates(lib, prec):
    """All-to-all register under S_128: 8 candidate pulses of one Hamiltonian (500 slices,
    65 blocks) in one plan; candidates 0 and 5 against oracle values stored by
    tests/golden/make_golden.py, and every candidate's norm against 1."""
    import torch
    print(f"S_128 candidates {prec}", flush=True)
    w = W.config5(seed=0, C=8)
    uc = w.notes["u_candidates"]
    rng = w.notes["rng"]
    B = lib.Basis(128, "symmetric")
    S = lib.System(B, w.h0, w.hk)
    D = B.dim
    states = []
    for _ in range(uc.shape[0]):
        vf = W.gaussian_panel(rng, D)
        v0 = W.gaussian_panel(rng, D)
        states.append((v0, vf))
    P = lib.Plan.batched([S] * uc.shape[0], prec, [w.N] * uc.shape[0], [w.dt] * uc.shape[0], 1.0)
    out, grads = lib.fidelity_grad_batched(P, [torch.tensor(u, device="cuda") for u in uc],
                                           [torch.tensor(s[0], device="cuda") for s in states],
                                           [torch.tensor(s[1], device="cuda") for s in states])
    tf = 1e-12 if prec == "c128" else 1e-6
    # |psi_N|^2 - 1: FP64 keeps it at rounding level; an FP32 propagator is unitary to about
    # 2e-7 per slice (the degree-12 evaluation), which can accumulate over the 500 slices
    # (F and the gradient are normalised by |psi_N|^2 and are held to tf below)
    tn = 1e-12 if prec == "c128" else 500 * 2e-7
    assert np.abs(out[:, 4].cpu().numpy() - 1.0).max() <= tn
    for c in (0, 5):
        vals, gref = read_golden(f"sym128_C8_cand{c}_N{w.N}.txt")
        g = grads[c].cpu().numpy()
        tg = 1e-12 if prec == "c128" else fp32_grad_tol(np.abs(gref).max())
        print(f"  candidate {c}: |dF|={abs(out[c, 0].item() - vals['F']):.2e} "
              f"max|dg|={np.abs(g - gref).max():.2e}", flush=True)
        assert abs(out[c, 0].item() - vals["F"]) <= tf
        assert np.abs(g - gref).max() <= tg


def test_progress_lines_per_problem_group(lib, capfd):
    """qoc_set_progress: one stderr line per finished problem group, from the call's stream."""
    import torch
    print("progress lines", flush=True)
    rng = np.random.default_rng(47)
    ws = []
    for n, N in ((8, 40), (6, 20), (8, 30), (7, 25)):
        u = rng.uniform(-1, 1, (N, 2))
        ws.append(W.Workload(f"ring{n}", n, "dihedral", 1, W.heisenberg_ring_terms(0.9), W.global_controls(), N,
                             0.04, u))
    states = [_problem_states(rng, w.n) for w in ws]
    systems = [lib.System(lib.Basis(w.n), w.h0, w.hk) for w in ws]
    Ns, dts = [w.N for w in ws], [w.dt for w in ws]
    full = lib.Plan.batched(systems, "c64", Ns, dts, 1.0).workspace_bytes
    Pg, frac = None, 0.5
    while frac > 0.01:
        cand = lib.Plan.batched(systems, "c64", Ns, dts, 1.0, int(full * frac))
        if cand.info["problem_groups"] >= 2:
            Pg = cand
            break
        frac *= 0.8
    assert Pg is not None
    G = Pg.info["problem_groups"]
    capfd.readouterr()
    lib.set_progress(True)
    try:
        lib.fidelity_grad_batched(Pg, [torch.tensor(w.u, device="cuda") for w in ws],
                                  [torch.tensor(s[0], device="cuda") for s in states],
                                  [torch.tensor(s[1], device="cuda") for s in states])
        torch.cuda.synchronize()
    finally:
        lib.set_progress(False)
    err = capfd.readouterr().err
    lines = [l for l in err.splitlines() if l.startswith("[qoc] problem group")]
    assert len(lines) == G and lines[-1].startswith(f"[qoc] problem group {G}/{G} done")


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_problem_groups_equal_the_single_group_plan(lib, prec):
    """A batched plan whose budget cannot hold every problem's propagators runs groups of
    problems one after another (no recompute): results bit for bit those of the plan that
    holds them all, for the full call, the objective-only call and the states read back; the
    FP64 results also against the oracle."""
    import torch
    print(f"problem groups {prec}", flush=True)
    rng = np.random.default_rng(41)
    ws = []
    for n, N in ((8, 60), (6, 25), (8, 33), (7, 50), (6, 12), (8, 41)):
        u = rng.uniform(-1, 1, (N, 2))
        ws.append(W.Workload(f"ring{n}", n, "dihedral", 1, W.heisenberg_ring_terms(0.6 + 0.05 * n),
                             W.global_controls(), N, 0.04, u))
    states = [_problem_states(rng, w.n) for w in ws]
    systems = [lib.System(lib.Basis(w.n), w.h0, w.hk) for w in ws]
    Ns, dts = [w.N for w in ws], [w.dt for w in ws]
    us = [torch.tensor(w.u, device="cuda") for w in ws]
    p0 = [torch.tensor(s[0], device="cuda") for s in states]
    pf = [torch.tensor(s[1], device="cuda") for s in states]
    P1 = lib.Plan.batched(systems, prec, Ns, dts, 1.0)
    assert P1.info["problem_groups"] == 1 and P1.info["segments"] == 1
    o1, g1 = lib.fidelity_grad_batched(P1, us, p0, pf)
    full = P1.workspace_bytes
    Pg, frac = None, 0.5
    while frac > 0.01:
        cand = lib.Plan.batched(systems, prec, Ns, dts, 1.0, int(full * frac))
        if cand.info["problem_groups"] >= 3:
            Pg = cand
            break
        frac *= 0.8
    assert Pg is not None
    print(f"  groups {Pg.groups()}", flush=True)
    assert Pg.workspace_bytes <= int(full * frac)
    og_, gg = lib.fidelity_grad_batched(Pg, us, p0, pf)
    # out[6], the largest squaring count, is taken over the problems that share a group
    assert torch.equal(og_[:, :6], o1[:, :6]) and torch.equal(og_[:, 7], o1[:, 7])
    for a, b in zip(gg, g1):
        assert torch.equal(a, b)
    assert torch.equal(lib.fidelity_batched(Pg, us, p0, pf)[:, :6], o1[:, :6])
    last = len(ws) - 1
    lib.fidelity_grad_batched(Pg, us, p0, pf)
    st_g = lib.read_state(Pg, "psi", ws[last].N, problem=last)
    lib.fidelity_grad_batched(P1, us, p0, pf)
    assert torch.equal(st_g, lib.read_state(P1, "psi", ws[last].N, problem=last))
    if prec == "c128":
        for p, w in enumerate(ws):
            ref = _oracle(w, *states[p])
            assert abs(og_[p, 0].item() - ref["F"]) <= 1e-12
            assert np.abs(gg[p].cpu().numpy() - ref["grad"]).max() <= 1e-12


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_products_formed_in_the_workspace(lib, prec):
    """Operator products formed at the start of every call in the workspace (the form a batch
    of distinct Hamiltonians too large to keep them takes): complex128 results bit for bit
    those of the plan whose systems keep their products (both formed by the same FP64 set-up
    products), complex64 ones (products formed in FP32) against the FP64 oracle; and the same
    form with problem groups, each group forming its own, bit for bit the one-group plan."""
    import torch
    print(f"workspace products {prec}", flush=True)
    rng = np.random.default_rng(43)
    ws = []
    for n, N in ((8, 30), (6, 21), (7, 26), (8, 17)):
        u = rng.uniform(-1, 1, (N, 2))
        ws.append(W.Workload(f"ring{n}", n, "dihedral", 1, W.heisenberg_ring_terms(0.55 + 0.05 * n),
                             W.global_controls(), N, 0.04, u))
    states = [_problem_states(rng, w.n) for w in ws]
    Ns, dts = [w.N for w in ws], [w.dt for w in ws]
    us = [torch.tensor(w.u, device="cuda") for w in ws]
    p0 = [torch.tensor(s[0], device="cuda") for s in states]
    pf = [torch.tensor(s[1], device="cuda") for s in states]
    sys_kept = [lib.System(lib.Basis(w.n), w.h0, w.hk) for w in ws]
    Pk = lib.Plan.batched(sys_kept, prec, Ns, dts, 1.0)
    assert Pk.info["products_in_workspace"] == 0 and Pk.info["powers_from_generator"] == 2
    ok, gk = lib.fidelity_grad_batched(Pk, us, p0, pf)
    lib.set_products_policy(1)
    try:
        sys_ws = [lib.System(lib.Basis(w.n), w.h0, w.hk) for w in ws]
        Pw = lib.Plan.batched(sys_ws, prec, Ns, dts, 1.0)
        full = Pw.workspace_bytes
        Pg, frac = None, 0.5
        while frac > 0.01:
            cand = lib.Plan.batched(sys_ws, prec, Ns, dts, 1.0, int(full * frac))
            if cand.info["problem_groups"] >= 3:
                Pg = cand
                break
            frac *= 0.8
    finally:
        lib.set_products_policy(0)
    assert Pw.info["products_in_workspace"] == 1 and Pw.info["powers_from_generator"] == 2
    assert Pw.workspace_bytes > Pk.workspace_bytes
    ow, gw = lib.fidelity_grad_batched(Pw, us, p0, pf)
    assert int(ow[:, 7].abs().max().item()) == 0
    assert Pg is not None and Pg.info["products_in_workspace"] == 1
    print(f"  groups {Pg.groups()}", flush=True)
    og_, gg = lib.fidelity_grad_batched(Pg, us, p0, pf)
    assert torch.equal(og_[:, :6], ow[:, :6])
    for a, b in zip(gg, gw):
        assert torch.equal(a, b)
    if prec == "c128":
        assert torch.equal(ow[:, :6], ok[:, :6])
        for a, b in zip(gw, gk):
            assert torch.equal(a, b)
    for p, w in enumerate(ws):
        ref = _oracle(w, *states[p])
        g = gw[p].cpu().numpy()
        tf = 1e-12 if prec == "c128" else 1e-6
        tg = 1e-12 if prec == "c128" else fp32_grad_tol(np.abs(ref["grad"]).max())
        assert abs(ow[p, 0].item() - ref["F"]) <= tf
        assert np.abs(g - ref["grad"]).max() <= tg
