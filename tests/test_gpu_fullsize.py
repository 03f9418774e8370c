"""Full-size workloads against the oracle.  The benchmark workload (12-qubit ring under D12,
9 blocks, 1000 slices) in the launch configuration bench.py times: all-blocks states vs the
oracle values stored by tests/golden/make_golden.py, and the plain variant (all-up to a
state of the first block) vs the SU(2) closed form computed here.  The 14-qubit ring with
staggered controls under the two-site group (blocks up to 2340 wide), first 8 slices of its
pulse, vs stored oracle values."""
import numpy as np
import pytest

import qoc_workloads as W
from oracle import basis as obasis
from oracle import closed_form
from tests._common import fp32_grad_tol, read_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ring12(lib):
    w = W.config2(seed=0, variant="all")
    B = lib.Basis(12, "dihedral", 1)
    S = lib.System(B, w.h0, w.hk)
    return w, B, S


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_allblocks_full_size_vs_oracle(lib, ring12, prec):
    import torch
    print(f"ring12 all blocks full size {prec}", flush=True)
    w, B, S = ring12
    # replay the input protocol: J, u, then psi_f and psi0 over all 4096 panel entries
    w2 = W.config2(seed=0, variant="all")
    rng = w2.notes["rng"]
    vf = W.gaussian_panel(rng, 4096)
    v0 = W.gaussian_panel(rng, 4096)
    vals, gref = read_golden("ring12_D12_allblocks_N1000.txt")
    P = lib.Plan(S, prec, w.N, w.dt, 2.0)  # the benchmark's plan
    out, grad = lib.fidelity_grad(P, torch.tensor(w.u, device="cuda"), torch.tensor(v0, device="cuda"),
                                  torch.tensor(vf, device="cuda"))
    F = out[0].item()
    g = grad.cpu().numpy()
    if prec == "c128":
        assert abs(F - vals["F"]) <= 1e-12
        assert np.abs(g - gref).max() <= 1e-12
    else:
        assert abs(F - vals["F"]) <= 1e-6
        assert np.abs(g - gref).max() <= fp32_grad_tol(np.abs(gref).max())
    print(f"  |dF| = {abs(F - vals['F']):.2e}  max|dg| = {np.abs(g - gref).max():.2e}", flush=True)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_plain_full_size_vs_closed_form(lib, ring12, prec):
    """All-up to a Gaussian state of the first block: F and the whole gradient equal the SU(2)
    product closed form (isotropic coupling contributes only a phase)."""
    import torch
    print(f"ring12 plain closed form {prec}", flush=True)
    w, B, S = ring12
    w2 = W.config2(seed=0, variant="plain")
    rng = w2.notes["rng"]
    m0 = B.sizes[0]
    pf = W.gaussian_panel(rng, m0)
    V, reps = obasis.convention_basis(12, "A1")
    psif_dense = V[0] @ pf
    ref = closed_form.fidelity_grad(12, 0.5, w2.J, [("x", 1.0), ("y", 1.0)], w2.u, w2.dt, psif_dense)
    v0 = np.zeros(4096, complex)
    v0[0] = 1.0
    vf = np.zeros(4096, complex)
    vf[:m0] = pf
    P = lib.Plan(S, prec, w2.N, w2.dt, 2.0)
    out, grad = lib.fidelity_grad(P, torch.tensor(w2.u, device="cuda"), torch.tensor(v0, device="cuda"),
                                  torch.tensor(vf, device="cuda"))
    g = grad.cpu().numpy()
    # one-basis-state start: the FP32 bound for such transfers (2.6e-5 max|g| measured)
    tf, tg = (1e-12, 1e-12) if prec == "c128" else (1e-6, fp32_grad_tol(np.abs(ref["grad"]).max(), 5e-5))
    dg = np.abs(g - ref["grad"]).max()
    print(f"  |dF| {abs(out[0].item() - ref['F']):.2e} max|dg| {dg:.2e} ({dg / np.abs(ref['grad']).max():.2e} of max|g|)",
          flush=True)
    assert abs(out[0].item() - ref["F"]) <= tf
    assert dg <= tg


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_ring14_two_site_group_vs_oracle(lib, prec):
    """Largest ring blocks (1300, 1044 and three 2340-wide E blocks, 4 controls): the first
    8 slices of the 14-qubit staggered-control pulse, every block carrying state."""
    import torch
    print(f"ring14 two-site group {prec}", flush=True)
    w = W.config4(seed=0, variant="all")
    rng = w.notes["rng"]
    B = lib.Basis(14, "dihedral", 2)
    S = lib.System(B, w.h0, w.hk)
    vf = W.gaussian_panel(rng, B.dim)
    v0 = W.gaussian_panel(rng, B.dim)
    vals, gref = read_golden("ring14_T2R_allblocks_N8.txt")
    N = gref.shape[0]
    P = lib.Plan(S, prec, N, w.dt, 2.0)
    out, grad = lib.fidelity_grad(P, torch.tensor(w.u[:N], device="cuda"), torch.tensor(v0, device="cuda"),
                                  torch.tensor(vf, device="cuda"))
    F = out[0].item()
    g = grad.cpu().numpy()
    print(f"  sizes {B.sizes}  |dF| = {abs(F - vals['F']):.2e}  max|dg| = {np.abs(g - gref).max():.2e}", flush=True)
    assert abs(out[4].item() - vals["normN2"]) <= (1e-12 if prec == "c128" else 1e-6)
    if prec == "c128":
        assert abs(F - vals["F"]) <= 1e-12
        assert np.abs(g - gref).max() <= 1e-12
    else:
        assert abs(F - vals["F"]) <= 1e-6
        assert np.abs(g - gref).max() <= fp32_grad_tol(np.abs(gref).max())


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_ring14_segmented_vs_oracle(lib, prec):
    """The 14-qubit two-site-group workload's first 64 slices on a plan whose workspace budget
    forces at least three segments (the 1300-2340-wide blocks swept co-operatively across
    segment boundaries, earlier segments recomputed in the backward sweep) against stored
    oracle values, and bit for bit the plan of the default budget (one segment when the free
    memory allows; complex128 blocks sweep one work-group each)."""
    import torch
    from tests._common import plan_with_segments
    print(f"ring14 segmented {prec}", flush=True)
    w = W.config4(seed=0, variant="all")
    rng = w.notes["rng"]
    B = lib.Basis(14, "dihedral", 2)
    S = lib.System(B, w.h0, w.hk)
    vf = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    v0 = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    vals, gref = read_golden("ring14_T2R_allblocks_N64.txt")
    N = gref.shape[0]
    u = torch.tensor(w.u[:N], device="cuda")
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    P1 = lib.Plan(S, prec, N, w.dt, 2.0)  # the default budget: one segment when memory allows
    o1, g1 = lib.fidelity_grad(P1, u, v0, vf)
    seg1 = P1.info["segments"]
    del P1
    torch.cuda.empty_cache()
    P = plan_with_segments(lib, S, prec, N, w.dt, 2.0, 3)
    print(f"  plan {P.info} (default-budget plan: {seg1} segments)", flush=True)
    assert P.info["segments"] >= 3
    # complex64: the co-operative sweep (64-row groups); complex128 blocks need more 32-row
    # groups than the CUs hold, so they sweep one work-group per block
    assert P.info["sweep_groups"] > 1 if prec == "c64" else P.info["sweep_groups"] == 1
    out, grad = lib.fidelity_grad(P, u, v0, vf)
    assert torch.equal(out[:6], o1[:6]) and torch.equal(grad, g1)
    g = grad.cpu().numpy()
    print(f"  |dF| = {abs(out[0].item() - vals['F']):.2e}  max|dg| = {np.abs(g - gref).max():.2e}", flush=True)
    if prec == "c128":
        assert abs(out[0].item() - vals["F"]) <= 1e-12
        assert np.abs(g - gref).max() <= 1e-12
    else:
        assert abs(out[0].item() - vals["F"]) <= 1e-6
        assert np.abs(g - gref).max() <= fp32_grad_tol(np.abs(gref).max())
