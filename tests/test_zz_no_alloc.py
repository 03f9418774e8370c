"""qoc_fidelity_grad_noalloc (workspace from the library's static device scratch, no
allocation in the call) against qoc_fidelity_grad with a caller workspace, through the C ABI:
two calls in a row, the second on a smaller problem, each bit for bit equal to the
workspace call; a plan whose workspace exceeds the static scratch is rejected."""
import ctypes

import numpy as np
import pytest

import qoc_workloads as W

pytestmark = pytest.mark.gpu


def _case(lib, n, N, seed, prec):
    import torch
    w = W.config2(seed=seed, N=N, n=n, variant="all")
    rng = np.random.default_rng(seed + 50)
    B = lib.Basis(n)
    S = lib.System(B, w.h0, w.hk)
    P = lib.Plan(S, prec, N, w.dt, 2.0, lib.STATIC_SCRATCH_BYTES)
    u = torch.tensor(w.u, device="cuda")
    p0 = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    pf = torch.tensor(W.gaussian_panel(rng, B.dim), device="cuda")
    return B, S, P, u, p0, pf


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_noalloc_matches_workspace_call(lib, prec):
    import torch
    from paper_2309_05884_amd import _capi as C
    print(f"no-alloc entry point {prec}", flush=True)
    cases = [(10, 300, 1), (8, 40, 2)]  # the second call is the smaller problem
    for n, N, seed in cases:
        B, S, P, u, p0, pf = _case(lib, n, N, seed, prec)
        assert P.workspace_bytes <= lib.STATIC_SCRATCH_BYTES
        ref_out, ref_grad = lib.fidelity_grad(P, u, p0, pf)
        out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
        grad = torch.full((N, P.K), float("nan"), dtype=torch.float64, device="cuda")
        st = C.lib().qoc_fidelity_grad_noalloc(P._h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(p0.data_ptr()),
                                               ctypes.c_void_p(pf.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                               ctypes.c_void_p(grad.data_ptr()),
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == 0, C.lib().qoc_last_error()
        torch.cuda.synchronize()
        print(f"  n={n} N={N} segments={P.info['segments']}: F {out[0].item():.15e} ref {ref_out[0].item():.15e}",
              flush=True)
        assert out[7].item() == 0
        assert torch.equal(out[:7], ref_out[:7])
        assert torch.equal(grad, ref_grad)


def test_noalloc_rejects_plans_beyond_the_static_scratch(lib):
    import torch
    print("no-alloc size limit", flush=True)
    w = W.config2(seed=0, N=1000, n=12, variant="all")
    B = lib.Basis(12)
    S = lib.System(B, w.h0, w.hk)
    P = lib.Plan(S, "c64", w.N, w.dt, 2.0)
    assert P.workspace_bytes > lib.STATIC_SCRATCH_BYTES
    u = torch.tensor(w.u, device="cuda")
    p = torch.zeros(B.dim, dtype=torch.complex128, device="cuda")
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    grad = torch.empty((w.N, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.QocError) as e:
        lib.fidelity_grad_noalloc(P, u, p, p, out, grad)
    assert e.value.status == 4
