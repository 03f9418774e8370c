"""The device gradient is the derivative of the device objective: central finite
differences (h = 1e-4, FP64 path) on every (slice, control) pair of the first 8 slices of
the 14-qubit ring with staggered controls under the two-site group (32 pairs: 8 slices x 4
controls), independent of the oracle."""
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
