"""GEMM tile variants and the autotuner: every variant gives bit-identical objective and
gradient (each output element accumulates over k in the same order), and autotuning keeps
one of them without changing results."""
import numpy as np
import pytest

import qoc_workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,n,N", [("c64", 12, 40), ("c128", 10, 24)])
def test_variants_identical_and_autotune(lib, prec, n, N):
    import torch
    print(f"GEMM variants {prec} n={n} N={N}", flush=True)
    w = W.config2(seed=0, variant="all") if n == 12 else None
    rng = np.random.default_rng(5)
    if w is None:
        w = W.Workload(f"ring{n}", n, "dihedral", 1, W.heisenberg_ring_terms(0.9), W.global_controls(), N, 0.02,
                       rng.uniform(-2, 2, (N, 2)))
    u = torch.tensor(np.ascontiguousarray(w.u[:N]), device="cuda")
    B = lib.Basis(n)
    S = lib.System(B, w.h0, w.hk)
    psif = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    psi0 = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    P = lib.Plan(S, prec, N, w.dt, 2.0)
    assert P.info["gemm_variant"] == 0
    ref_o, ref_g = (t.clone() for t in lib.fidelity_grad(P, u, psi0, psif))
    for v in range(P.N_VARIANTS):
        P.set_variant(v)
        assert P.info["gemm_variant"] == v
        o, g = lib.fidelity_grad(P, u, psi0, psif)
        print(f"  variant {v} ({P.variant_name}): equal {torch.equal(o, ref_o) and torch.equal(g, ref_g)}", flush=True)
        assert torch.equal(o, ref_o) and torch.equal(g, ref_g)
    chosen, times = P.autotune(u)
    print(f"  autotune -> {chosen} ({P.variant_name}), ms {[round(t, 3) for t in times]}", flush=True)
    assert 0 <= chosen < P.N_VARIANTS and P.info["gemm_variant"] == chosen
    assert all(t > 0 for t in times) and times[chosen] == min(times)
    o, g = lib.fidelity_grad(P, u, psi0, psif)
    assert torch.equal(o, ref_o) and torch.equal(g, ref_g)
