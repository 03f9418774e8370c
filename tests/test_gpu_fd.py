"""The device gradient is the derivative of the device objective: central finite
differences (h = 1e-4, FP64 path) on every (slice, control) pair of the first 8 slices of
the 14-qubit ring with staggered controls under the two-site group (32 pairs: 8 slices x 4
controls), independent of the oracle; and, at the workload's full size (4000 slices), on 32
seeded pairs through the slice-local identity, with sampled outputs against the oracle."""
import os

import numpy as np
import pytest

import qoc_workloads as W

pytestmark = pytest.mark.gpu


def test_central_differences_ring14(lib):
    import torch
    print("central differences ring14 two-site group", flush=True)
    w = W.config4(seed=0, variant="all")
    rng = w.notes["rng"]
    N, h = 8, 1e-4
    B = lib.Basis(14, "dihedral", 2)
    S = lib.System(B, w.h0, w.hk)
    vf = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    v0 = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    P = lib.Plan(S, "c128", N, w.dt, 2.0)
    u = torch.tensor(w.u[:N], device="cuda")
    out, grad = lib.fidelity_grad(P, u, v0, vf)
    g = grad.cpu().numpy()
    fd = np.zeros_like(g)
    for j in range(N):
        for k in range(u.shape[1]):
            up, um = u.clone(), u.clone()
            up[j, k] += h
            um[j, k] -= h
            fp = lib.fidelity_grad(P, up, v0, vf)[0][0].item()
            fm = lib.fidelity_grad(P, um, v0, vf)[0][0].item()
            fd[j, k] = (fp - fm) / (2 * h)
    err = np.abs(fd - g).max()
    print(f"  F {out[0].item():.6e}  max|g| {np.abs(g).max():.3e}  max|fd - g| {err:.2e}", flush=True)
    # central-difference truncation h^2 F'''/6 and FP64 rounding of F (~1e-16 / h) are both
    # far below this bound; the gradient entries are O(1e-6)
    assert err <= 1e-9 + 1e-4 * np.abs(g).max()


FULL = os.environ.get("QOC_FULL_SIZE_TESTS") == "1"


@pytest.mark.skipif(not FULL, reason="full-size 4000-slice run (about 5 GPU-minutes): set QOC_FULL_SIZE_TESTS=1")
def test_ring14_full_pulse_fd_and_invariants(lib):
    """The 14-qubit staggered-control workload at its full size: 4000 slices of 0.01, all
    blocks (1300, 1044, 3 x 2340) of the two-site group, complex128, with the default
    workspace budget (segments recomputed in the backward sweep).  Checked on outputs the
    oracle can compute one by one and on properties that hold at any size:
    * o_j = <psi_f|psi_j> for j = 8 and 64 against the oracle's objective of the first j
      slices (stored values);
    * o = <lambda_j|psi_j> at sampled j;
    * central differences (h = 1e-4) of F on 32 seeded (slice, control) pairs spread over the
      pulse, through the slice-local identity o(u + h e_jk) = <lambda_{j+1}|U_j(u')|psi_j>
      (only slice j changes), against the gradient;
    * the complex64 plan of the same pulse: |dF| <= 1e-6 and gradient within fp32_grad_tol of
      the complex128 one."""
    import torch
    from tests._common import fp32_grad_tol, read_golden
    print("ring14 full pulse, complex128", flush=True)
    w = W.config4(seed=0, variant="all")
    rng = w.notes["rng"]
    N, h = w.N, 1e-4
    B = lib.Basis(14, "dihedral", 2)
    S = lib.System(B, w.h0, w.hk)
    vf = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    v0 = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    u = torch.tensor(w.u, device="cuda")
    P = lib.Plan(S, "c128", N, w.dt, 2.0)
    print(f"  plan {P.info}", flush=True)
    out, grad = lib.fidelity_grad(P, u, v0, vf)
    torch.cuda.synchronize()
    o = complex(out[2].item(), out[3].item())
    g = grad.cpu().numpy()
    print(f"  F {out[0].item():.15e} segments {P.info['segments']}", flush=True)
    vfn = vf.cpu().numpy()
    for j in (8, 64):
        name = f"ring14_T2R_allblocks_N{j}.txt"
        vals, _ = read_golden(name)
        oj = np.vdot(vfn, lib.read_state(P, "psi", j).cpu().numpy())
        print(f"  o_{j} {oj:.15e} oracle {vals['o_re']:.15e}{vals['o_im']:+.15e}j", flush=True)
        assert abs(oj - complex(vals["o_re"], vals["o_im"])) <= 1e-12
    for j in (1, 777, 2048, 3999, N):
        lam = lib.read_state(P, "lambda", j).cpu().numpy()
        psi = lib.read_state(P, "psi", j).cpu().numpy()
        assert abs(np.vdot(lam, psi) - o) <= 1e-12 * max(1.0, abs(o)), j
    pick = np.random.default_rng(4000)
    pairs = sorted(set((int(j), int(k)) for j, k in zip(pick.integers(0, N, 40), pick.integers(0, 4, 40))))[:32]
    P1 = lib.Plan(S, "c128", 1, w.dt, 2.0 + 2 * h)
    norms = out[4].item() * out[5].item()
    worst = 0.0
    for (j, k) in pairs:
        psi_j = lib.read_state(P, "psi", j)
        lam_j1 = lib.read_state(P, "lambda", j + 1)
        vals = []
        for sgn in (1.0, -1.0):
            uj = u[j:j + 1].clone()
            uj[0, k] += sgn * h
            vals.append(lib.fidelity(P1, uj, psi_j, lam_j1)[1].item())
        fd = (vals[0] - vals[1]) / (2 * h) / norms
        worst = max(worst, abs(fd - g[j, k]))
    print(f"  FD on {len(pairs)} pairs: max|fd - g| {worst:.2e}, max|g| {np.abs(g).max():.2e}", flush=True)
    assert worst <= 1e-9 + 1e-4 * np.abs(g).max()
    del P, P1
    torch.cuda.empty_cache()
    print("ring14 full pulse, complex64", flush=True)
    P32 = lib.Plan(S, "c64", N, w.dt, 2.0)
    out32, grad32 = lib.fidelity_grad(P32, u, v0, vf)
    dF = abs(out32[0].item() - out[0].item())
    dg = np.abs(grad32.cpu().numpy() - g).max()
    print(f"  |dF| {dF:.2e} max|dg| {dg:.2e} ({dg / np.abs(g).max():.2e} of max|g|)", flush=True)
    # F ~ 3e-6 after the 4000 slices: max|g| (2.5e-6) is small against the costates' rounding
    # scale 2 |o| dt ||H_k|| u32 sqrt(N) ~ 2e-9, so the absolute floor of fp32_grad_tol binds
    # (measured 1.9e-10)
    assert dF <= 1e-6 and dg <= fp32_grad_tol(np.abs(g).max())
