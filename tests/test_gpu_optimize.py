"""The library's L-BFGS GRAPE optimiser (qoc_optimize_lbfgs) against the oracle's
(oracle/optimize.py) on the same seeded problem: the transfer all-up -> all-down in the
first D_n block of a nearest-neighbour Ising ring (Eq. (5)) under global controls
(Eq. (6)).  In complex128 both follow the same accepted steps, so the F histories, the
number of evaluations, the stop reason and the final controls agree; in complex64 the
result is re-evaluated by the FP64 oracle."""
import numpy as np
import pytest

import qoc_workloads as W
from oracle import grape
from oracle import optimize as opt

pytestmark = pytest.mark.gpu

N_QUBITS, N, DT = 5, 30, 0.05
REASON = {opt.TARGET: "target", opt.GTOL: "gtol", opt.MAX_ITER: "max_iter",
          opt.LINE_SEARCH_FAILED: "line_search_failed"}


def _problem(seed):
    n = N_QUBITS
    h0, hk = W.ising_ring_terms(1.0, 1.0), W.global_controls(0.5)
    blocks = grape.block_system(n, h0, hk)
    up = np.zeros(2 ** n, complex)
    up[0] = 1.0
    dn = np.zeros(2 ** n, complex)
    dn[-1] = 1.0
    p0 = grape.panels_from_dense(blocks, up)[:1]
    pf = grape.panels_from_dense(blocks, dn)[:1]
    rng = np.random.default_rng(seed)
    t = (np.arange(N) + 0.5) * DT
    u0 = rng.uniform(-0.3, 0.3, (N, 2))
    u0[:, 0] += 0.25 * np.cos(t)
    u0[:, 1] += 0.25 * np.sin(t)
    return h0, hk, blocks[:1], p0, pf, u0


def _gpu_plan(lib, h0, hk, prec, u_bound):
    B = lib.Basis(N_QUBITS, "dihedral", 1)
    S = lib.System(B, h0, hk)
    return lib.Plan(S, prec, N, DT, u_bound, blocks=[0])


@pytest.mark.parametrize("u_bound", [3.0, 0.6])
def test_c128_optimiser_follows_the_oracle(lib, u_bound):
    import torch
    print(f"optimiser parity c128 u_bound={u_bound}", flush=True)
    h0, hk, b0, p0, pf, u0 = _problem(21)
    kw = dict(memory=5, step0=0.3, c1=1e-4, max_backtrack=12, max_iter=25, f_target=1.0, gtol=0.0)
    ref = opt.lbfgs_ascent(opt.grape_objective(b0, DT, p0, pf, (N, 2), u_bound=u_bound), u0.reshape(-1), **kw)
    P = _gpu_plan(lib, h0, hk, "c128", u_bound)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda")
    got = lib.optimize_lbfgs(P, dev(u0), dev(p0[0].ravel()), dev(pf[0].ravel()), **kw)
    print(f"  oracle {ref['hist'][-1]:.12f} ({len(ref['hist'])} points, {ref['evals']} evals, "
          f"{REASON[ref['reason']]}); library {got['F']:.12f} ({len(got['hist'])}, {got['evaluations']}, "
          f"{got['reason']})", flush=True)
    assert ref["hist"][-1] > 10 * ref["hist"][0]  # the run does optimise
    assert got["evaluations"] == ref["evals"] and got["reason"] == REASON[ref["reason"]]
    assert len(got["hist"]) == len(ref["hist"])
    assert np.abs(got["hist"] - ref["hist"]).max() <= 1e-10
    assert abs(got["F"] - ref["F"]) <= 1e-10
    assert np.abs(got["u"].cpu().numpy().reshape(-1) - ref["u"]).max() <= 1e-8 * max(1.0, np.abs(ref["u"]).max())


def test_c64_optimiser_reaches_target_confirmed_in_fp64(lib):
    import torch
    print("optimiser c64 to F >= 0.9", flush=True)
    h0, hk, b0, p0, pf, u0 = _problem(22)
    P = _gpu_plan(lib, h0, hk, "c64", 3.0)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda")
    got = lib.optimize_lbfgs(P, dev(u0), dev(p0[0].ravel()), dev(pf[0].ravel()), memory=8, step0=0.3,
                             max_iter=200, f_target=0.9)
    print(f"  {got['reason']} after {got['iterations']} steps, {got['evaluations']} evals, F {got['F']:.8f}",
          flush=True)
    assert got["reason"] == "target" and got["F"] >= 0.9
    assert np.all(np.diff(got["hist"]) >= 0.0)
    u = got["u"].cpu().numpy()
    F64 = grape.fidelity_grad(b0, u, DT, p0, pf)["F"]
    assert abs(F64 - got["F"]) <= 1e-5


def test_optimiser_argument_errors(lib):
    import torch
    from paper_2309_05884_amd._capi import QocError
    h0, hk, b0, p0, pf, u0 = _problem(23)
    P = _gpu_plan(lib, h0, hk, "c128", 0.6)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda")
    a, b = dev(p0[0].ravel()), dev(pf[0].ravel())
    with pytest.raises(QocError, match="INVALID_ARG"):
        lib.optimize_lbfgs(P, dev(u0), a, b, memory=0)
    with pytest.raises(QocError, match="INVALID_ARG"):
        lib.optimize_lbfgs(P, dev(u0), a, b, c1=1.5)
    with pytest.raises(QocError, match="NUMERIC"):  # start outside the plan's norm bound
        lib.optimize_lbfgs(P, dev(np.full((N, 2), 5.0)), a, b)
    Bd = lib.Basis(N_QUBITS, "dihedral", 1)
    S = lib.System(Bd, h0, hk)
    PB = lib.Plan.batched([S, S], "c128", [N, N], [DT, DT], 1.0)
    import ctypes
    from paper_2309_05884_amd import _capi as C
    nbytes = ctypes.c_size_t()
    assert C.lib().qoc_optimize_workspace_size(PB._h, 4, ctypes.byref(nbytes)) == 3  # unsupported
    # max_iter = 0: the start is evaluated and returned unchanged
    r = lib.optimize_lbfgs(P, dev(u0), a, b, max_iter=0)
    assert r["reason"] == "max_iter" and r["iterations"] == 0 and r["evaluations"] == 1
    assert np.array_equal(r["u"].cpu().numpy(), u0)
    F0 = grape.fidelity_grad(b0, u0, DT, p0, pf)["F"]
    assert abs(r["F"] - F0) <= 1e-12


def test_optimiser_on_a_segmented_plan_takes_the_same_steps(lib):
    """A workspace budget that holds only part of the propagators makes the plan recompute
    segments in the backward sweep; the optimiser's steps are unchanged (the recomputed
    propagators are the same arithmetic)."""
    import torch
    print("optimiser segmented plan", flush=True)
    h0, hk, b0, p0, pf, u0 = _problem(24)
    P = _gpu_plan(lib, h0, hk, "c128", 3.0)
    Pseg = None
    for frac in (0.6, 0.45, 0.3, 0.2, 0.14, 0.1, 0.07, 0.05):
        B = lib.Basis(N_QUBITS, "dihedral", 1)
        S = lib.System(B, h0, hk)
        cand = lib.Plan(S, "c128", N, DT, 3.0, max_workspace_bytes=int(P.workspace_bytes * frac), blocks=[0])
        if cand.info["segments"] > 1:
            Pseg = cand
            break
    assert Pseg is not None
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda")
    kw = dict(memory=5, step0=0.3, max_iter=10, f_target=1.0)
    a = lib.optimize_lbfgs(P, dev(u0), dev(p0[0].ravel()), dev(pf[0].ravel()), **kw)
    b = lib.optimize_lbfgs(Pseg, dev(u0), dev(p0[0].ravel()), dev(pf[0].ravel()), **kw)
    assert a["evaluations"] == b["evaluations"] and np.array_equal(a["hist"], b["hist"])
    assert torch.equal(a["u"], b["u"])


def test_trotterised_optimiser_follows_the_oracle(lib):
    """GRAPE with per-qubit controls through the Trotterised propagator
    (qoc_optimize_lbfgs_lts) takes the oracle's L-BFGS steps on the oracle's Trotterised
    objective and gradient (oracle/lts.py)."""
    import torch
    from oracle import lts
    print("optimiser, Trotterised per-qubit controls", flush=True)
    n, Nn, dt, Bz, c = 4, 20, 0.1, 1.0, 1.0
    rng = np.random.default_rng(25)
    u0 = rng.uniform(-0.3, 0.3, (Nn, 2 * n))
    p0 = np.zeros(2 ** n, complex)
    p0[0] = 1.0
    pf = np.zeros(2 ** n, complex)
    pf[-1] = 1.0

    def fun(uf):
        r = lts.fidelity_grad(n, Bz, c, uf.reshape(Nn, 2 * n), dt, p0, pf)
        return r["F"], r["grad"].reshape(-1), bool(np.isfinite(r["F"]))

    kw = dict(memory=6, step0=0.5, c1=1e-4, max_backtrack=12, max_iter=15, f_target=1.0, gtol=0.0)
    ref = opt.lbfgs_ascent(fun, u0.reshape(-1), **kw)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda")
    got = lib.optimize_lbfgs_lts(n, Bz, c, dev(u0), dt, dev(p0), dev(pf), **kw)
    print(f"  oracle F {ref['F']:.12f} ({ref['evals']} evals); library F {got['F']:.12f} "
          f"({got['evaluations']} evals)", flush=True)
    assert ref["hist"][-1] > 10 * ref["hist"][0]
    assert got["evaluations"] == ref["evals"] and got["reason"] == REASON[ref["reason"]]
    assert np.abs(got["hist"] - ref["hist"]).max() <= 1e-10
    assert np.abs(got["u"].cpu().numpy().reshape(-1) - ref["u"]).max() <= 1e-8 * max(1.0, np.abs(ref["u"]).max())
