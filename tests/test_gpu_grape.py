"""Objective and exact gradient on the device (Eqs. (3)-(4); App. B) against the FP64 oracle.

Tolerances: FP64 |dF| <= 1e-12 and gradient error <= 1e-12 (absolute; gradients are
O(1e-2)); FP32: |dF| <= 1e-6 and gradient error <= 2e-5 * max|g| (tests/_common.py gives the
derivation), from FP32 rounding of U_j (relative ~1e-7 per slice, growing like sqrt(N))
entering the costates."""
import numpy as np
import pytest

import qoc_workloads as W
from oracle import grape as og
from tests._common import all_states, flat_from_panels, fp32_grad_tol, oracle_blocks, plain_states, plan_with_segments

pytestmark = pytest.mark.gpu


def _device(lib, n, group, stride, h0, hk, u, dt, psi0, psif, prec, max_ws=0, u_bound=None):
    import torch
    B = lib.Basis(n, group, stride)
    S = lib.System(B, h0, hk)
    ub = float(np.abs(u).max()) if u_bound is None else u_bound
    P = lib.Plan(S, prec, u.shape[0], dt, ub, max_ws)
    out, grad = lib.fidelity_grad(P, torch.tensor(u, device="cuda"),
                                  torch.tensor(flat_from_panels(psi0), device="cuda"),
                                  torch.tensor(flat_from_panels(psif), device="cuda"))
    torch.cuda.synchronize()
    return out.cpu().numpy(), grad.cpu().numpy(), P


def _tol(prec, g, rel=None):
    if prec == "c128":
        return 1e-12, 1e-12
    return 1e-6, fp32_grad_tol(np.abs(g).max()) if rel is None else fp32_grad_tol(np.abs(g).max(), rel)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_config1_plain(lib, prec):
    print(f"config1 plain {prec}", flush=True)
    w = W.config1()
    ob = oracle_blocks(6, w.h0, w.hk)
    psi0, psif = plain_states(ob, w.notes["rng"])
    ref = og.fidelity_grad(ob, w.u, w.dt, psi0, psif)
    out, grad, P = _device(lib, 6, "dihedral", 1, w.h0, w.hk, w.u, w.dt, psi0, psif, prec)
    tf, tg = _tol(prec, ref["grad"], 5e-5)  # one-basis-state start (tests/_common.py)
    assert abs(out[0] - ref["F"]) <= tf
    assert abs(out[1] - ref["F_raw"]) <= tf
    assert np.abs(grad - ref["grad"]).max() <= tg
    assert out[7] == 0


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_all_blocks_full_coupling(lib, prec):
    """Non-degenerate dynamics in every block: Eq. (7) couplings plus a Heisenberg ring."""
    print(f"all blocks full coupling {prec}", flush=True)
    n = 7
    h0 = W.full_coupling_terms(n, 1.0, [0.3, 0.17, 0.11]) + [W.ring_pair(0.4, "xx"), W.ring_pair(0.4, "yy")]
    hk = [[W.one_body(0.5, "x")], [W.one_body(0.5, "y")]]
    rng = np.random.default_rng(21)
    u = rng.uniform(-1.5, 1.5, (64, 2))
    ob = oracle_blocks(n, h0, hk)
    psi0, psif = all_states(ob, rng)
    ref = og.fidelity_grad(ob, u, 0.05, psi0, psif)
    out, grad, P = _device(lib, n, "dihedral", 1, h0, hk, u, 0.05, psi0, psif, prec)
    tf, tg = _tol(prec, ref["grad"])
    assert abs(out[0] - ref["F"]) <= tf
    assert np.abs(grad - ref["grad"]).max() <= tg


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_generator_split_is_bitwise_neutral(lib, prec):
    """The slice generator over its automatic number of column ranges, one range and three
    (qoc_plan_set_generator_split) gives the same objective and gradient bit for bit; the
    automatic one against the oracle."""
    import torch
    print(f"generator split {prec}", flush=True)
    n, N, dt = 10, 240, 0.02
    h0, hk = W.heisenberg_ring_terms(1.0), W.global_controls()
    rng = np.random.default_rng(31)
    u = rng.uniform(-1.0, 1.0, (N, 2))
    ob = oracle_blocks(n, h0, hk)
    assert max(b["H0"].shape[0] for b in ob) >= 64  # wide enough for the split to apply
    psi0, psif = all_states(ob, rng)
    B = lib.Basis(n, "dihedral", 1)
    P = lib.Plan(lib.System(B, h0, hk), prec, N, dt, 1.0)
    args = (torch.tensor(u, device="cuda"), torch.tensor(flat_from_panels(psi0), device="cuda"),
            torch.tensor(flat_from_panels(psif), device="cuda"))
    res = []
    for k in (0, 1, 3):
        P.set_generator_split(k)
        out, grad = lib.fidelity_grad(P, *args)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy().copy(), grad.cpu().numpy().copy()))
    for out, grad in res[1:]:
        assert np.array_equal(out[:6], res[0][0][:6])
        assert np.array_equal(grad, res[0][1])
    ref = og.fidelity_grad(ob, u, dt, psi0, psif)
    tf, tg = _tol(prec, ref["grad"])
    assert abs(res[0][0][0] - ref["F"]) <= tf
    assert np.abs(res[0][1] - ref["grad"]).max() <= tg
    with pytest.raises(lib.QocError):
        P.set_generator_split(-1)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_two_site_group_four_controls(lib, prec):
    """The staggered-control workload (K = 4) under the two-site rotation group."""
    print(f"two-site group {prec}", flush=True)
    n = 8
    w = W.config4(N=40, n=n)
    rng = np.random.default_rng(5)
    ob = oracle_blocks(n, w.h0, w.hk, "dihedral", 2)
    psi0, psif = all_states(ob, rng)
    ref = og.fidelity_grad(ob, w.u, w.dt * 3, psi0, psif)
    out, grad, P = _device(lib, n, "dihedral", 2, w.h0, w.hk, w.u, w.dt * 3, psi0, psif, prec)
    tf, tg = _tol(prec, ref["grad"])
    assert abs(out[0] - ref["F"]) <= tf
    assert np.abs(grad - ref["grad"]).max() <= tg


def test_symmetric_group_blocks(lib):
    print("symmetric group", flush=True)
    n = 6
    h0 = [W.one_body(1.0, "z"), W.all_pairs(0.2, "xx"), W.all_pairs(0.1, "yy")]
    hk = [[W.one_body(1.0, "x")], [W.one_body(1.0, "y")]]
    rng = np.random.default_rng(9)
    u = rng.uniform(-1, 1, (30, 2))
    ob = og.block_system(n, h0, hk, "symmetric")
    psi0, psif = all_states(ob, rng)
    ref = og.fidelity_grad(ob, u, 0.05, psi0, psif)
    out, grad, P = _device(lib, n, "symmetric", 1, h0, hk, u, 0.05, psi0, psif, "c128")
    assert abs(out[0] - ref["F"]) <= 1e-12
    assert np.abs(grad - ref["grad"]).max() <= 1e-12


def test_large_norm_substeps(lib):
    """dt large enough for squarings and Frechet sub-steps (R > 1)."""
    print("large norm substeps", flush=True)
    w = W.config1(N=12)
    ob = oracle_blocks(6, w.h0, w.hk)
    rng = np.random.default_rng(2)
    psi0, psif = all_states(ob, rng)
    ref = og.fidelity_grad(ob, w.u, 0.5, psi0, psif)
    out, grad, P = _device(lib, 6, "dihedral", 1, w.h0, w.hk, w.u, 0.5, psi0, psif, "c128")
    assert P.info["substeps"] > 1 and P.info["max_squarings"] >= 1
    assert abs(out[0] - ref["F"]) <= 1e-12
    assert np.abs(grad - ref["grad"]).max() <= 1e-11


def test_segmented_recompute_matches(lib):
    """A workspace too small for all propagators forces segments and recomputation."""
    print("segmented recompute", flush=True)
    w = W.config1(N=50)
    ob = oracle_blocks(6, w.h0, w.hk)
    psi0, psif = all_states(ob, np.random.default_rng(4))
    ref = og.fidelity_grad(ob, w.u, w.dt, psi0, psif)
    out1, g1, P1 = _device(lib, 6, "dihedral", 1, w.h0, w.hk, w.u, w.dt, psi0, psif, "c128")
    small = plan_with_segments(lib, P1.system, "c128", w.N, w.dt, float(np.abs(w.u).max())).workspace_bytes
    out2, g2, P2 = _device(lib, 6, "dihedral", 1, w.h0, w.hk, w.u, w.dt, psi0, psif, "c128", max_ws=small)
    assert P2.info["segments"] > 1
    assert abs(out2[0] - ref["F"]) <= 1e-12
    assert np.abs(g2 - ref["grad"]).max() <= 1e-12
    assert np.array_equal(out1[:6], out2[:6])


def test_deterministic_and_edge_cases(lib):
    import torch
    print("determinism, N=1, u=0", flush=True)
    w = W.config1(N=20)
    ob = oracle_blocks(6, w.h0, w.hk)
    psi0, psif = all_states(ob, np.random.default_rng(8))
    o1, g1, _ = _device(lib, 6, "dihedral", 1, w.h0, w.hk, w.u, w.dt, psi0, psif, "c128")
    o2, g2, _ = _device(lib, 6, "dihedral", 1, w.h0, w.hk, w.u, w.dt, psi0, psif, "c128")
    assert np.array_equal(o1, o2) and np.array_equal(g1, g2)
    for u in (w.u[:1], np.zeros((5, 2))):
        ref = og.fidelity_grad(ob, u, w.dt, psi0, psif)
        o, g, _ = _device(lib, 6, "dihedral", 1, w.h0, w.hk, u, w.dt, psi0, psif, "c128", u_bound=1.0)
        assert abs(o[0] - ref["F"]) <= 1e-12
        assert np.abs(g - ref["grad"]).max() <= 1e-12


def test_control_beyond_bound_is_reported(lib):
    import torch
    w = W.config1(N=10)
    ob = oracle_blocks(6, w.h0, w.hk)
    psi0, psif = all_states(ob, np.random.default_rng(1))
    with pytest.raises(lib.QocError) as e:
        _device(lib, 6, "dihedral", 1, w.h0, w.hk, 3 * w.u, w.dt, psi0, psif, "c128", u_bound=0.5)
    assert e.value.status == 6


def test_autograd_function(lib):
    import torch
    print("autograd", flush=True)
    w = W.config1(N=30)
    ob = oracle_blocks(6, w.h0, w.hk)
    psi0, psif = plain_states(ob, np.random.default_rng(0))
    ref = og.fidelity_grad(ob, w.u, w.dt, psi0, psif)
    B = lib.Basis(6)
    S = lib.System(B, w.h0, w.hk)
    P = lib.Plan(S, "c128", 30, w.dt, 1.0)
    u = torch.tensor(w.u, device="cuda", requires_grad=True)
    F = lib.GrapeFidelity.apply(u, P, torch.tensor(flat_from_panels(psi0), device="cuda"),
                                torch.tensor(flat_from_panels(psif), device="cuda"))
    (3.0 * F).backward()
    assert abs(F.item() - ref["F"]) <= 1e-12
    assert np.abs(u.grad.cpu().numpy() - 3.0 * ref["grad"]).max() <= 3e-12


def test_workspace_budgets_bitwise_equal(lib):
    """Smaller workspaces form the propagators in chunks of slices (Taylor scratch for one
    chunk) and then in segments recomputed during the backward sweep; every budget gives
    the same objective and gradient bit for bit."""
    print("workspace budgets", flush=True)
    w = W.config1(N=48)
    ob = oracle_blocks(6, w.h0, w.hk)
    psi0, psif = all_states(ob, np.random.default_rng(6))
    out1, g1, P1 = _device(lib, 6, "dihedral", 1, w.h0, w.hk, w.u, w.dt, psi0, psif, "c64")
    assert P1.info["segments"] == 1 and P1.info["expm_chunk"] == 48 and P1.info["propagator_planes"] == 4
    full = P1.workspace_bytes
    seen = set()
    for frac in (0.9, 0.75, 0.5, 0.35, 0.25, 0.18, 0.12, 0.08):
        o, g, P = _device(lib, 6, "dihedral", 1, w.h0, w.hk, w.u, w.dt, psi0, psif, "c64", max_ws=int(full * frac))
        info = P.info
        seen.add((info["segments"] > 1, info["expm_chunk"] < info["segment"]))
        print(f"  budget {frac}: segments {info['segments']} segment {info['segment']} chunk {info['expm_chunk']} "
              f"planes {info['propagator_planes']}", flush=True)
        assert np.array_equal(o[:6], out1[:6]) and np.array_equal(g, g1)
        if info["segments"] > 1:
            break
    assert (False, True) in seen or (True, True) in seen
    assert any(seg for seg, _ in seen)
