"""Segmented recompute (propagators of earlier segments formed again during the backward
sweep) on blocks whose sweeps split over several work-groups, against stored oracle values;
the co-operative sweep's solo fallback and its stall handling, forced from the host.

Bounds: FP64 |dF| and |d grad| <= 1e-12; FP32 |dF| <= 1e-6 and |d grad| <= 2e-5 max|g|
(the FP32 gradient error measured on these workloads is 4e-6 max|g|)."""
import numpy as np
import pytest

import qoc_workloads as W
from tests._common import plan_with_segments, read_golden

pytestmark = pytest.mark.gpu


def _ring12(lib):
    import torch
    w = W.config2(seed=0, variant="all")
    rng = w.notes["rng"]
    B = lib.Basis(12, "dihedral", 1)
    S = lib.System(B, w.h0, w.hk)
    vf = W.gaussian_panel(rng, B.dim)
    v0 = W.gaussian_panel(rng, B.dim)
    dev = (torch.tensor(w.u, device="cuda"), torch.tensor(v0, device="cuda"), torch.tensor(vf, device="cuda"))
    return w, B, S, dev


def _ring14(lib, N):
    import torch
    w = W.config4(seed=0, variant="all")
    rng = w.notes["rng"]
    B = lib.Basis(14, "dihedral", 2)
    S = lib.System(B, w.h0, w.hk)
    vf = W.gaussian_panel(rng, B.dim)
    v0 = W.gaussian_panel(rng, B.dim)
    dev = (torch.tensor(w.u[:N], device="cuda"), torch.tensor(v0, device="cuda"), torch.tensor(vf, device="cuda"))
    return w, B, S, dev


def _check(prec, out, grad, vals, gref):
    dF = abs(out[0] - vals["F"])
    dg = np.abs(grad - gref).max()
    gmax = np.abs(gref).max()
    print(f"  |dF| {dF:.2e}  max|dg| {dg:.2e} ({dg / gmax:.2e} of max|g|)", flush=True)
    if prec == "c128":
        assert dF <= 1e-12 and dg <= 1e-12
    else:
        assert dF <= 1e-6 and dg <= 2e-5 * gmax


def test_ring12_segmented_cooperative_matches_oracle(lib):
    """12-qubit ring, all 9 blocks (128-346 wide: 2-6 work-groups per block in the FP32
    sweeps), 1000 slices, a budget that forces at least 3 segments: the stored oracle values
    to the FP32 bounds, and bit for bit the one-segment plan's results."""
    import torch
    print("ring12 segmented, co-operative sweeps", flush=True)
    w, B, S, (u, v0, vf) = _ring12(lib)
    vals, gref = read_golden("ring12_D12_allblocks_N1000.txt")
    P1 = lib.Plan(S, "c64", w.N, w.dt, 2.0)
    assert P1.info["segments"] == 1 and P1.info["sweep_groups"] > 1
    o1, g1 = lib.fidelity_grad(P1, u, v0, vf)
    o1, g1 = o1.cpu().numpy(), g1.cpu().numpy()
    del P1
    torch.cuda.empty_cache()
    P = plan_with_segments(lib, S, "c64", w.N, w.dt, 2.0, 3)
    print(f"  plan {P.info}", flush=True)
    assert P.info["sweep_groups"] > 1
    o, g = lib.fidelity_grad(P, u, v0, vf)
    o, g = o.cpu().numpy(), g.cpu().numpy()
    _check("c64", o, g, vals, gref)
    assert np.array_equal(o[:6], o1[:6]) and np.array_equal(g, g1)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_ring14_two_site_group_segmented(lib, prec):
    """The 14-qubit staggered-control workload under the two-site group (blocks 1300, 1044,
    3 x 2340; too many rows for both sweeps' work-groups to share the CUs, so each block is
    swept by one work-group), first 8 slices, segments of at most 3 slices: every backward
    segment but the last recomputes 1300-2340-wide propagators.  Against the stored oracle
    values."""
    import torch
    print(f"ring14 segmented {prec}", flush=True)
    N = 8
    w, B, S, (u, v0, vf) = _ring14(lib, N)
    vals, gref = read_golden(f"ring14_T2R_allblocks_N{N}.txt")
    P = plan_with_segments(lib, S, prec, N, w.dt, 2.0, 3, budget_frac=0.4)
    print(f"  plan {P.info}", flush=True)
    o, g = lib.fidelity_grad(P, u, v0, vf)
    _check(prec, o.cpu().numpy(), g.cpu().numpy(), vals, gref)
    del P
    torch.cuda.empty_cache()


def test_forced_solo_sweeps(lib):
    """The co-operative sweep's fallback (one work-group runs a multi-group block alone)
    forced from the host: FP32 ring-12 against the stored oracle values, and FP64 on a
    10-qubit ring against the oracle run here."""
    import torch
    from oracle import grape as og
    from tests._common import all_states, flat_from_panels, oracle_blocks
    print("forced solo sweeps", flush=True)
    w, B, S, (u, v0, vf) = _ring12(lib)
    vals, gref = read_golden("ring12_D12_allblocks_N1000.txt")
    P = lib.Plan(S, "c64", w.N, w.dt, 2.0)
    assert P.info["sweep_groups"] > 1
    P.set_sweep_mode(lib.SWEEP_SOLO)
    o, g = lib.fidelity_grad(P, u, v0, vf)
    _check("c64", o.cpu().numpy(), g.cpu().numpy(), vals, gref)
    del P
    torch.cuda.empty_cache()
    n = 10
    w10 = W.config2(seed=3, N=60, n=n, variant="all")
    ob = oracle_blocks(n, w10.h0, w10.hk)
    psi0, psif = all_states(ob, np.random.default_rng(12))
    ref = og.fidelity_grad(ob, w10.u, w10.dt, psi0, psif)
    B10 = lib.Basis(n)
    S10 = lib.System(B10, w10.h0, w10.hk)
    for mode in (0, lib.SWEEP_SOLO):
        P10 = lib.Plan(S10, "c128", w10.N, w10.dt, 2.0)
        assert P10.info["sweep_groups"] > 1
        P10.set_sweep_mode(mode)
        o, g = lib.fidelity_grad(P10, torch.tensor(w10.u, device="cuda"),
                                 torch.tensor(flat_from_panels(psi0), device="cuda"),
                                 torch.tensor(flat_from_panels(psif), device="cuda"))
        assert abs(o[0].item() - ref["F"]) <= 1e-12
        assert np.abs(g.cpu().numpy() - ref["grad"]).max() <= 1e-12


@pytest.mark.parametrize("stall,segmented", [("fwd", False), ("bwd", False), ("bwd", True)])
def test_sweep_stall_is_reported(lib, stall, segmented):
    """A co-operative hand-off that never arrives (forced from the host: the groups wait for
    tags nobody writes, each wait bounded) must surface as status bit 2 and QocError, on the
    one-segment plan and after the backward sweeps of a segmented plan."""
    import torch
    print(f"sweep stall {stall} segmented={segmented}", flush=True)
    w, B, S, (u, v0, vf) = _ring12(lib)
    N = 64
    u = u[:N].contiguous()
    P = plan_with_segments(lib, S, "c64", N, w.dt, 2.0, 3) if segmented else lib.Plan(S, "c64", N, w.dt, 2.0)
    assert P.info["sweep_groups"] > 1
    P.set_sweep_mode(lib.SWEEP_TEST_STALL_FWD if stall == "fwd" else lib.SWEEP_TEST_STALL_BWD)
    out, _ = lib.fidelity_grad(P, u, v0, vf, check=False)
    flags = int(out[7].item())
    assert flags & 4, flags
    with pytest.raises(lib.QocError) as e:
        lib.check_flags(out)
    assert e.value.status == 6
    # the same plan runs cleanly again once the switch is off
    P.set_sweep_mode(0)
    out, _ = lib.fidelity_grad(P, u, v0, vf)
    assert int(out[7].item()) == 0
