"""Symmetry-reduced GRAPE on AMD Instinct MI355X (gfx950).

Thin Python layer over the C ABI of ``include/qoc.h``: it marshals arguments, takes
device memory and the current stream from PyTorch, and raises on error.  Every step
of the computation runs in the HIP library ``libqoc_gfx950.so``; there is no CPU
fallback, and importing the compute entry points without the built library fails.

Method: Wang, Okyay, Kumar & Wong, AVS Quantum Sci. 2023 -- block diagonalisation of
ring (D_n) and permutation (S_n) symmetric Hamiltonians (Sec. II A, App. A), slice
propagators (Eq. (3)), the state-transfer objective (Eq. (4)) and its gradient
(App. B, Eq. (B2), taken exactly).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _capi as C
from ._capi import QocError

__all__ = ["Basis", "System", "Plan", "fidelity_grad", "fidelity_grad_batched", "fidelity", "fidelity_batched",
           "read_state", "check_flags", "measure_mfma_peak", "fidelity_grad_noalloc", "STATIC_SCRATCH_BYTES", "propagate", "GrapeFidelity", "SWEEP_SOLO", "SWEEP_TEST_STALL_FWD", "SWEEP_TEST_STALL_BWD",
           "QocError", "library_path", "set_progress", "set_products_policy", "profile_begin", "profile_end", "slice_stats", "CapturedStep",
           "optimize_lbfgs", "gate_propagate", "gate_fidelity", "lts_apply",
           "lts_fidelity_grad", "optimize_lbfgs_lts"]

library_path = C.LIB_PATH

# co-operative sweep switches of qoc_plan_set_sweep_mode (tests of the fallback and of the
# stall handling; 0 in normal use)
SWEEP_SOLO, SWEEP_TEST_STALL_FWD, SWEEP_TEST_STALL_BWD = 1, 2, 4
# size of the library's static device scratch (QOC_STATIC_SCRATCH_BYTES): the largest plan
# workspace qoc_fidelity_grad_noalloc accepts
STATIC_SCRATCH_BYTES = 64 << 20


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Basis:
    """Orbits and block table of a group acting on n qubits (qoc_build_basis)."""

    def __init__(self, n: int, group: str = "dihedral", stride: int = 1):
        self._h = ctypes.c_void_p()
        L = C.lib()
        C.check(L.qoc_build_basis(int(n), C.GROUPS[group], int(stride), _stream(), ctypes.byref(self._h)))
        self.n, self.group, self.stride = n, group, stride
        nb = ctypes.c_int()
        C.check(L.qoc_basis_blocks(self._h, ctypes.byref(nb), None, None, 0))
        sizes = (ctypes.c_int32 * nb.value)()
        copies = (ctypes.c_int32 * nb.value)()
        C.check(L.qoc_basis_blocks(self._h, ctypes.byref(nb), sizes, copies, nb.value))
        self.sizes = [int(v) for v in sizes]
        self.copies = [int(v) for v in copies]

    @property
    def dim(self):
        return sum(m * d for m, d in zip(self.sizes, self.copies))

    def reps(self, which: int) -> np.ndarray:
        """which = 0: group orbits, 1: rotation orbits, 2 + b: representatives of block b."""
        L = C.lib()
        cnt = ctypes.c_int64()
        C.check(L.qoc_basis_reps(self._h, int(which), None, 0, ctypes.byref(cnt)))
        out = np.zeros(cnt.value, dtype=np.uint64)
        C.check(L.qoc_basis_reps(self._h, int(which), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                 cnt.value, ctypes.byref(cnt)))
        return out

    def to_blocks(self, dense):
        torch = _torch()
        dense = dense.to(torch.complex128).contiguous()
        out = torch.empty(self.dim, dtype=torch.complex128, device=dense.device)
        C.check(C.lib().qoc_state_to_blocks(self._h, _ptr(dense), _ptr(out), _stream()))
        return out

    def from_blocks(self, panel):
        torch = _torch()
        panel = panel.to(torch.complex128).contiguous()
        out = torch.empty(2 ** self.n, dtype=torch.complex128, device=panel.device)
        C.check(C.lib().qoc_state_from_blocks(self._h, _ptr(panel), _ptr(out), _stream()))
        return out

    def __del__(self):
        if getattr(self, "_h", None) and C._lib is not None:
            C._lib.qoc_basis_free(self._h)
            self._h = None


class System:
    """H0 and the control Hamiltonians projected into every block (qoc_project)."""

    def __init__(self, basis: Basis, h0_terms, hk_terms):
        self.basis = basis  # keeps the basis alive
        self.K = len(hk_terms)
        h0 = C.make_terms(h0_terms)
        flat = [t for lst in hk_terms for t in lst]
        hk = C.make_terms(flat)
        nhk = (ctypes.c_int * max(1, self.K))(*[len(l) for l in hk_terms])
        self._h = ctypes.c_void_p()
        C.check(C.lib().qoc_project(basis._h, h0, len(h0_terms), hk, nhk, self.K, _stream(), ctypes.byref(self._h)))

    def block(self, b: int, op: int):
        torch = _torch()
        m = self.basis.sizes[b]
        out = torch.empty((m, m), dtype=torch.complex128, device="cuda")
        C.check(C.lib().qoc_system_block(self._h, int(b), int(op), _ptr(out), _stream()))
        # the library writes column-major: transpose the row-major view
        return out.t().contiguous()

    def __del__(self):
        if getattr(self, "_h", None) and C._lib is not None:
            C._lib.qoc_system_free(self._h)
            self._h = None


class Plan:
    """Execution plan (qoc_plan_create / qoc_plan_create_batched).

    ``Plan(system, precision, N, dt, u_bound)`` plans one problem; ``blocks=[i, ...]`` limits
    it to those blocks of the system (qoc_plan_create_blocks; panels then hold only them).
    ``Plan.batched(systems, precision, Ns, dts, u_bound)`` plans several independent
    problems that share every launch (systems may repeat, e.g. one Hamiltonian with many
    candidate pulses)."""

    INFO_KEYS = ["segment", "segments", "taylor_step", "max_degree", "series_terms", "substeps",
                 "bytes_per_slice", "max_squarings", "grad_chunk", "gemm_grid", "problems", "jobs",
                 "total_controls", "total_panel", "total_propagator", "gemm_variant", "expm_chunk", "sweep_groups",
                 "problem_groups", "powers_from_generator", "propagator_planes",
                 "products_in_workspace"]
    N_VARIANTS = 3

    def __init__(self, system: System, precision: str = "c128", N: int = 1, dt: float = 0.01,
                 u_bound: float = 1.0, max_workspace_bytes: int = 0, _batch=None, blocks=None):
        self.precision, self.u_bound = precision, float(u_bound)
        self._h = ctypes.c_void_p()
        self.blocks = None if blocks is None else [int(b) for b in blocks]
        if _batch is None and self.blocks is not None:
            self.systems, self.Ns, self.dts = [system], [int(N)], [float(dt)]
            arr = (ctypes.c_int * len(self.blocks))(*self.blocks)
            C.check(C.lib().qoc_plan_create_blocks(system._h, arr, len(self.blocks), C.PRECISIONS[precision], int(N),
                                                   float(dt), float(u_bound), int(max_workspace_bytes),
                                                   ctypes.byref(self._h)))
        elif _batch is None:
            self.systems, self.Ns, self.dts = [system], [int(N)], [float(dt)]
            C.check(C.lib().qoc_plan_create(system._h, C.PRECISIONS[precision], int(N), float(dt), float(u_bound),
                                            int(max_workspace_bytes), ctypes.byref(self._h)))
        else:
            self.systems, self.Ns, self.dts = _batch
            P = len(self.systems)
            arr = (ctypes.c_void_p * P)(*[s_._h.value for s_ in self.systems])
            Ns = (ctypes.c_int * P)(*self.Ns)
            dts = (ctypes.c_double * P)(*self.dts)
            C.check(C.lib().qoc_plan_create_batched(arr, P, Ns, dts, C.PRECISIONS[precision], float(u_bound),
                                                    int(max_workspace_bytes), ctypes.byref(self._h)))
        self.system = self.systems[0]
        self.N, self.dt, self.K = self.Ns[0], self.dts[0], self.systems[0].K
        self.Ks = [s_.K for s_ in self.systems]
        self.P = len(self.systems)
        b = ctypes.c_size_t()
        C.check(C.lib().qoc_plan_workspace_size(self._h, ctypes.byref(b)))
        self.workspace_bytes = int(b.value)
        self._ws = None
        self._refresh_info()

    def _refresh_info(self):
        n = len(self.INFO_KEYS)
        info = (ctypes.c_int64 * n)()
        C.check(C.lib().qoc_plan_info(self._h, info, n))
        self.info = dict(zip(self.INFO_KEYS, [int(v) for v in info]))

    @property
    def variant_name(self):
        return C.lib().qoc_variant_name(C.PRECISIONS[self.precision], self.info["gemm_variant"]).decode()

    def set_variant(self, v: int):
        """Use GEMM tile variant v (0..N_VARIANTS-1); results do not change."""
        C.check(C.lib().qoc_plan_set_variant(self._h, int(v)))
        self._refresh_info()

    def autotune(self, u):
        """Time every GEMM tile variant on this plan's work for controls u (device tensor,
        concatenated for a batch) and keep the fastest; returns (chosen, [ms per variant])."""
        torch = _torch()
        u = u.to(torch.float64).contiguous().reshape(-1)
        ws = self.workspace()
        chosen = ctypes.c_int()
        times = (ctypes.c_double * self.N_VARIANTS)()
        C.check(C.lib().qoc_plan_autotune(self._h, _ptr(u), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(),
                                          ctypes.byref(chosen), times))
        self._refresh_info()
        return int(chosen.value), [float(t) for t in times]

    @classmethod
    def batched(cls, systems, precision="c64", Ns=None, dts=None, u_bound=1.0, max_workspace_bytes=0):
        systems = list(systems)
        return cls(None, precision, u_bound=u_bound, max_workspace_bytes=max_workspace_bytes,
                   _batch=(systems, [int(n) for n in Ns], [float(d) for d in dts]))

    def block_sizes(self):
        """Block sizes m of a one-problem plan, in plan order (the subset when blocks= was given)."""
        sizes = self.systems[0].basis.sizes
        return list(sizes) if self.blocks is None else [sizes[b] for b in self.blocks]

    def groups(self):
        """Problem groups (qoc_plan_groups): [(first problem, segment length, segments)]."""
        L = C.lib()
        n = ctypes.c_int()
        C.check(L.qoc_plan_groups(self._h, ctypes.byref(n), None, None, None, 0))
        b0 = (ctypes.c_int32 * n.value)()
        sl = (ctypes.c_int32 * n.value)()
        ns = (ctypes.c_int32 * n.value)()
        C.check(L.qoc_plan_groups(self._h, ctypes.byref(n), b0, sl, ns, n.value))
        return [(int(b0[g]), int(sl[g]), int(ns[g])) for g in range(n.value)]

    def set_sweep_mode(self, mode: int):
        """Co-operative sweep switches (SWEEP_SOLO, SWEEP_TEST_STALL_FWD / _BWD bits; 0 = normal)."""
        C.check(C.lib().qoc_plan_set_sweep_mode(self._h, int(mode)))

    def set_generator_split(self, ranges: int):
        """Generator column ranges (qoc_plan_set_generator_split): 0 = automatic, k >= 1 = k
        ranges (capped by the widest block); results are the same bit for bit."""
        C.check(C.lib().qoc_plan_set_generator_split(self._h, int(ranges)))

    def workspace(self):
        torch = _torch()
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device="cuda")
        return self._ws

    def __del__(self):
        if getattr(self, "_h", None) and C._lib is not None:
            C._lib.qoc_plan_free(self._h)
            self._h = None


PROFILE_KINDS = ["generator", "propagator_gemm", "gate_chain", "sweep_fwd", "sweep_bwd", "objective",
                 "gradient_gemm", "gradient_vector", "gradient_finish", "other"]


def measure_mfma_peak(precision: str = "c64") -> float:
    """Measured TFLOP/s of the matrix-core instruction the tiles use (qoc_measure_mfma_peak)."""
    v = ctypes.c_double()
    C.check(C.lib().qoc_measure_mfma_peak(C.PRECISIONS[precision], ctypes.byref(v), _stream()))
    return float(v.value)


def set_products_policy(policy: int = 0):
    """Where new plans keep operator products: 0 automatic, 1 always in the workspace (qoc_set_products_policy)."""
    C.check(C.lib().qoc_set_products_policy(int(policy)))


def set_progress(enable: bool = True):
    """Per-group progress lines on stderr for calls on plans with problem groups (qoc_set_progress)."""
    C.check(C.lib().qoc_set_progress(1 if enable else 0))


def profile_begin(max_launches: int = 100000):
    """Start recording HIP events around every hot-path kernel launch (benchmarks only)."""
    C.check(C.lib().qoc_profile_begin(int(max_launches)))


def profile_end():
    """Stop recording; {kind: (total_ms, launches)} over the recorded launches."""
    ms = (ctypes.c_double * 10)()
    cnt = (ctypes.c_int64 * 10)()
    C.check(C.lib().qoc_profile_end(ms, cnt, 10))
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(PROFILE_KINDS)}


def slice_stats(plan: "Plan", u):
    """(q, s, norm) arrays of shape (jobs, max N): the propagators' evaluation (q >= 1:
    Paterson-Stockmeyer degree q r; q = 0: the four-product degree-12 scheme; -1 beyond a
    problem's N), squarings and FP64 norm."""
    torch = _torch()
    u = u.to(torch.float64).contiguous()
    nb = plan.info["jobs"]
    Nmax = max(plan.Ns)
    q = np.zeros((nb, Nmax), dtype=np.int32)
    s = np.zeros((nb, Nmax), dtype=np.int32)
    nrm = np.zeros((nb, Nmax), dtype=np.float64)
    C.check(C.lib().qoc_plan_slice_stats(plan._h, _ptr(u), q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         nrm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()))
    return q, s, nrm


def check_flags(out):
    """Raise if the objective's status word (out[7]) reports a numeric problem (synchronises)."""
    flags = int(out[7].item())
    if flags:
        what = []
        if flags & 1:
            what.append("a slice exceeded the plan's norm bound (|u| > u_bound)")
        if flags & 2:
            what.append("non-finite value")
        if flags & 4:
            what.append("a co-operative sweep stalled and gave up (outputs invalid)")
        raise QocError(6, "; ".join(what))


def _run(plan, u_flat, psi0_flat, psif_flat, workspace, check):
    torch = _torch()
    ws = workspace if workspace is not None else plan.workspace()
    out = torch.empty((plan.P, 8), dtype=torch.float64, device=u_flat.device)
    grad = torch.empty(plan.info["total_controls"], dtype=torch.float64, device=u_flat.device)
    C.check(C.lib().qoc_fidelity_grad(plan._h, _ptr(u_flat), _ptr(psi0_flat), _ptr(psif_flat), _ptr(out),
                                      _ptr(grad), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream()))
    if check:
        for p in range(plan.P):
            check_flags(out[p])
    return out, grad


def fidelity_grad(plan: Plan, u, psi0, psif, workspace=None, check=True):
    """(out[8], grad[N,K]) on the device for a one-problem plan: out = [F, |o|^2, Re o, Im o,
    |psi_N|^2, |psi_f|^2, max squarings, flags]."""
    torch = _torch()
    assert plan.P == 1
    u = u.to(torch.float64).contiguous()
    assert u.shape == (plan.N, plan.K) and u.is_cuda
    psi0 = psi0.to(torch.complex128).contiguous()
    psif = psif.to(torch.complex128).contiguous()
    D = plan.info["total_panel"]
    assert psi0.numel() == D and psif.numel() == D
    out, grad = _run(plan, u.reshape(-1), psi0, psif, workspace, check)
    return out[0], grad.view(plan.N, plan.K)


def _run_objective(plan, u_flat, psi0_flat, psif_flat, workspace, check):
    torch = _torch()
    ws = workspace if workspace is not None else plan.workspace()
    out = torch.empty((plan.P, 8), dtype=torch.float64, device=u_flat.device)
    C.check(C.lib().qoc_fidelity(plan._h, _ptr(u_flat), _ptr(psi0_flat), _ptr(psif_flat), _ptr(out), _ptr(ws),
                                 ctypes.c_size_t(ws.numel()), _stream()))
    if check:
        for p in range(plan.P):
            check_flags(out[p])
    return out


def fidelity(plan: Plan, u, psi0, psif, workspace=None, check=True):
    """Objective only (qoc_fidelity: propagators, forward sweep, overlap; no gradient) for a
    one-problem plan: out[8] as fidelity_grad returns it."""
    torch = _torch()
    assert plan.P == 1
    u = u.to(torch.float64).contiguous()
    assert u.shape == (plan.N, plan.K) and u.is_cuda
    psi0 = psi0.to(torch.complex128).contiguous()
    psif = psif.to(torch.complex128).contiguous()
    D = plan.info["total_panel"]
    assert psi0.numel() == D and psif.numel() == D
    return _run_objective(plan, u.reshape(-1), psi0, psif, workspace, check)[0]


def fidelity_batched(plan: Plan, us, psi0s, psifs, workspace=None, check=True):
    """Objective only for a batched plan: out[P, 8]."""
    torch = _torch()
    assert len(us) == plan.P == len(psi0s) == len(psifs)
    u_flat = torch.cat([u.to(torch.float64).reshape(-1) for u in us]).contiguous()
    p0 = torch.cat([v.to(torch.complex128).reshape(-1) for v in psi0s]).contiguous()
    pf = torch.cat([v.to(torch.complex128).reshape(-1) for v in psifs]).contiguous()
    assert u_flat.numel() == plan.info["total_controls"] and p0.numel() == plan.info["total_panel"]
    return _run_objective(plan, u_flat, p0, pf, workspace, check)


def read_state(plan: Plan, which: str, j: int, problem: int = 0, workspace=None):
    """A state of the last call's sweeps (qoc_plan_read_state): which = "psi" for psi_j
    (0 <= j <= N) or "lambda" for the costate lambda_j (1 <= j <= N), as block panels of
    problem `problem` (complex128 device tensor).  The workspace must be the one that call
    used (default: the plan's own)."""
    torch = _torch()
    ws = workspace if workspace is not None else plan.workspace()
    sizes = plan.systems[problem].basis.sizes
    copies = plan.systems[problem].basis.copies
    idx = range(len(sizes)) if plan.blocks is None else plan.blocks
    D = sum(sizes[b] * copies[b] for b in idx)
    out = torch.empty(D, dtype=torch.complex128, device="cuda")
    C.check(C.lib().qoc_plan_read_state(plan._h, int(problem), {"psi": 0, "lambda": 1}[which], int(j), _ptr(ws),
                                        ctypes.c_size_t(ws.numel()), _ptr(out), _stream()))
    return out


def fidelity_grad_noalloc(plan: Plan, u, psi0, psif, out, grad):
    """qoc_fidelity_grad_noalloc: objective and gradient of a one-problem plan with the
    library's static device scratch as workspace (the call allocates nothing).  out (8
    float64) and grad (N, K float64) are caller-allocated device tensors, written in place;
    u, psi0 and psif must already be contiguous device tensors of the right dtype."""
    torch = _torch()
    assert plan.P == 1
    assert u.dtype == torch.float64 and u.is_contiguous() and u.shape == (plan.N, plan.K)
    assert psi0.dtype == torch.complex128 and psif.dtype == torch.complex128
    assert psi0.is_contiguous() and psif.is_contiguous()
    assert psi0.numel() == plan.info["total_panel"] == psif.numel()
    assert out.dtype == torch.float64 and out.numel() >= 8 and out.is_contiguous()
    assert grad.dtype == torch.float64 and grad.numel() == plan.N * plan.K and grad.is_contiguous()
    C.check(C.lib().qoc_fidelity_grad_noalloc(plan._h, _ptr(u), _ptr(psi0), _ptr(psif), _ptr(out), _ptr(grad),
                                              _stream()))
    return out, grad


def fidelity_grad_batched(plan: Plan, us, psi0s, psifs, workspace=None, check=True):
    """Batched form: lists of per-problem controls (N_p, K_p) and panels; returns
    (out[P, 8], [grad_p (N_p, K_p)])."""
    torch = _torch()
    assert len(us) == plan.P == len(psi0s) == len(psifs)
    u_flat = torch.cat([u.to(torch.float64).reshape(-1) for u in us]).contiguous()
    p0 = torch.cat([v.to(torch.complex128).reshape(-1) for v in psi0s]).contiguous()
    pf = torch.cat([v.to(torch.complex128).reshape(-1) for v in psifs]).contiguous()
    assert u_flat.numel() == plan.info["total_controls"] and p0.numel() == plan.info["total_panel"]
    out, grad = _run(plan, u_flat, p0, pf, workspace, check)
    grads, off = [], 0
    for N, K in zip(plan.Ns, plan.Ks):
        grads.append(grad[off:off + N * K].view(N, K))
        off += N * K
    return out, grads


def propagate(plan: Plan, u, workspace=None):
    """Slice propagators U_j of every block (one-problem plan): list of (N, m, m) complex128
    tensors.  For a batched plan pass the concatenated controls; the result is one list per
    problem."""
    torch = _torch()
    u = u.to(torch.float64).contiguous().reshape(-1)
    ws = workspace if workspace is not None else plan.workspace()
    flat = torch.empty(plan.info["total_propagator"], dtype=torch.complex128, device=u.device)
    C.check(C.lib().qoc_propagate(plan._h, _ptr(u), _ptr(flat), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream()))
    per_problem, off = [], 0
    for sys_, N in zip(plan.systems, plan.Ns):
        outs = []
        sizes = sys_.basis.sizes if plan.blocks is None else [sys_.basis.sizes[b] for b in plan.blocks]
        for m in sizes:
            outs.append(flat[off:off + N * m * m].view(N, m, m).transpose(1, 2))  # column-major
            off += N * m * m
        per_problem.append(outs)
    return per_problem[0] if plan.P == 1 else per_problem


def gate_propagate(plan: Plan, u, workspace=None):
    """K = U_{N-1} ... U_0 of every block of a one-problem plan (qoc_gate_propagate): list of
    (m, m) complex128 device tensors in block order."""
    torch = _torch()
    assert plan.P == 1
    u = u.to(torch.float64).contiguous()
    assert u.shape == (plan.N, plan.K) and u.is_cuda
    ws = workspace if workspace is not None else plan.workspace()
    sizes = plan.block_sizes()
    flat = torch.empty(sum(m * m for m in sizes), dtype=torch.complex128, device=u.device)
    C.check(C.lib().qoc_gate_propagate(plan._h, _ptr(u), _ptr(flat), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                       _stream()))
    out, off = [], 0
    for m in sizes:
        out.append(flat[off:off + m * m].view(m, m).transpose(0, 1))  # column-major
        off += m * m
    return out


def gate_fidelity(plan: Plan, Ka, Kb, workspace=None):
    """Gate fidelity on the device (qoc_gate_fidelity) for block lists as gate_propagate
    returns: out = [F, Re t, Im t, D, na, nb], t = sum_blocks d Tr(Ka^dag Kb),
    F = |t|^2 / (na nb) with na, nb the weighted squared Frobenius norms (= D for
    unitaries)."""
    torch = _torch()

    def flat(Ks):
        return torch.cat([k.transpose(0, 1).contiguous().reshape(-1) for k in Ks]).to(torch.complex128).contiguous()

    a, b = flat(Ka), flat(Kb)
    assert a.numel() == b.numel() == sum(m * m for m in plan.block_sizes())
    ws = workspace if workspace is not None else plan.workspace()
    out = torch.empty(6, dtype=torch.float64, device=a.device)
    C.check(C.lib().qoc_gate_fidelity(plan._h, _ptr(a), _ptr(b), _ptr(out), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                      _stream()))
    return out


def lts_apply(n: int, Bz: float, c_cpl: float, u, dt: float, psi=None, ncols=None):
    """Trotterised per-qubit-control propagation (qoc_lts_apply): U_{N-1}^LTS ... U_0^LTS
    applied to the columns of psi (2^n x k complex128, computational basis), or, with
    psi=None, to the identity columns 0 .. ncols-1 (default all: K^LTS).  u: (N, 2n) with
    u[j, 2(i-1)] = Bx_i, u[j, 2(i-1)+1] = By_i.  Returns a (2^n, k) device tensor."""
    torch = _torch()
    u = u.to(torch.float64).contiguous()
    N = u.shape[0]
    assert u.shape == (N, 2 * n) and u.is_cuda
    D = 1 << n
    if psi is not None:
        psi = psi.to(torch.complex128)
        if psi.dim() == 1:
            psi = psi[:, None]
        assert psi.shape[0] == D
        k = psi.shape[1]
        src = psi.transpose(0, 1).contiguous()  # column-major
    else:
        k = D if ncols is None else int(ncols)
        src = None
    L = C.lib()
    nbytes = ctypes.c_size_t()
    C.check(L.qoc_lts_workspace_size(int(n), int(N), ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=u.device)
    out = torch.empty((k, D), dtype=torch.complex128, device=u.device)
    C.check(L.qoc_lts_apply(int(n), float(Bz), float(c_cpl), _ptr(u), int(N), float(dt),
                            None if src is None else _ptr(src), int(k), _ptr(out), _ptr(ws),
                            ctypes.c_size_t(ws.numel()), _stream()))
    return out.transpose(0, 1)


def lts_fidelity_grad(n: int, Bz: float, c_cpl: float, u, dt: float, psi0, psif):
    """Objective and exact gradient through the Trotterised per-qubit-control propagator
    (qoc_lts_fidelity_grad).  u: (N, 2n) or (P, N, 2n); psi0, psif: (2^n,) or (P, 2^n)
    complex128.  Returns (out (P, 8) or (8,), grad shaped like u) on the device."""
    torch = _torch()
    u = u.to(torch.float64).contiguous()
    single = u.dim() == 2
    if single:
        u = u[None]
    P, N = u.shape[0], u.shape[1]
    assert u.shape[2] == 2 * n and u.is_cuda
    D = 1 << n
    p0 = psi0.to(torch.complex128).reshape(P, D).contiguous()
    pf = psif.to(torch.complex128).reshape(P, D).contiguous()
    L = C.lib()
    nbytes = ctypes.c_size_t()
    C.check(L.qoc_lts_grad_workspace_size(int(n), int(N), int(P), ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=u.device)
    out = torch.empty((P, 8), dtype=torch.float64, device=u.device)
    grad = torch.empty_like(u)
    C.check(L.qoc_lts_fidelity_grad(int(n), float(Bz), float(c_cpl), _ptr(u), int(N), float(dt), int(P), _ptr(p0),
                                    _ptr(pf), _ptr(out), _ptr(grad), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                    _stream()))
    return (out[0], grad[0]) if single else (out, grad)


def optimize_lbfgs(plan: Plan, u, psi0, psif, max_iter=100, memory=10, step0=0.1, c1=1e-4,
                   max_backtrack=20, f_target=1.0, gtol=0.0):
    """GRAPE optimisation of a one-problem plan's controls by L-BFGS ascent with an Armijo
    line search (qoc_optimize_lbfgs).  Returns a dict: u (the last accepted controls,
    (N, K) on the device), F, hist (F at the start and after every accepted step),
    iterations, evaluations and reason ("target", "gtol", "max_iter",
    "line_search_failed")."""
    torch = _torch()
    assert plan.P == 1
    u = u.to(torch.float64).contiguous().clone()
    assert u.shape == (plan.N, plan.K) and u.is_cuda
    psi0 = psi0.to(torch.complex128).contiguous()
    psif = psif.to(torch.complex128).contiguous()
    D = plan.info["total_panel"]
    assert psi0.numel() == D and psif.numel() == D
    L = C.lib()
    nbytes = ctypes.c_size_t()
    C.check(L.qoc_optimize_workspace_size(plan._h, int(memory), ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=u.device)
    opts = C.QocLbfgsOptions(int(max_iter), int(memory), float(step0), float(c1), int(max_backtrack),
                             float(f_target), float(gtol))
    hist = (ctypes.c_double * (int(max_iter) + 1))()
    res = C.QocLbfgsResult()
    C.check(L.qoc_optimize_lbfgs(plan._h, ctypes.byref(opts), _ptr(u), _ptr(psi0), _ptr(psif), _ptr(ws),
                                 ctypes.c_size_t(ws.numel()), _stream(), hist, int(max_iter) + 1,
                                 ctypes.byref(res)))
    return {"u": u, "F": res.F, "hist": np.array(hist[:res.iterations + 1]), "iterations": res.iterations,
            "evaluations": res.evaluations, "reason": C.OPT_REASONS[res.reason]}


def optimize_lbfgs_lts(n: int, Bz: float, c_cpl: float, u, dt: float, psi0, psif, max_iter=100, memory=10,
                       step0=0.1, c1=1e-4, max_backtrack=20, f_target=1.0, gtol=0.0):
    """GRAPE through the Trotterised per-qubit-control propagator (qoc_optimize_lbfgs_lts):
    L-BFGS ascent on F(u), u of shape (N, 2n).  Returns a dict as optimize_lbfgs."""
    torch = _torch()
    u = u.to(torch.float64).contiguous().clone()
    N = u.shape[0]
    assert u.shape == (N, 2 * n) and u.is_cuda
    D = 1 << n
    psi0 = psi0.to(torch.complex128).reshape(D).contiguous()
    psif = psif.to(torch.complex128).reshape(D).contiguous()
    L = C.lib()
    nbytes = ctypes.c_size_t()
    C.check(L.qoc_optimize_lts_workspace_size(int(n), int(N), int(memory), ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=u.device)
    opts = C.QocLbfgsOptions(int(max_iter), int(memory), float(step0), float(c1), int(max_backtrack),
                             float(f_target), float(gtol))
    hist = (ctypes.c_double * (int(max_iter) + 1))()
    res = C.QocLbfgsResult()
    C.check(L.qoc_optimize_lbfgs_lts(int(n), float(Bz), float(c_cpl), int(N), float(dt), ctypes.byref(opts), _ptr(u),
                                     _ptr(psi0), _ptr(psif), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(), hist,
                                     int(max_iter) + 1, ctypes.byref(res)))
    return {"u": u, "F": res.F, "hist": np.array(hist[:res.iterations + 1]), "iterations": res.iterations,
            "evaluations": res.evaluations, "reason": C.OPT_REASONS[res.reason]}


class CapturedStep:
    """The whole hot path (propagators, both sweeps, objective, gradient) captured once into
    a HIP graph and replayed.  Inputs are read from, and outputs written to, the tensors
    given at capture time; copy new controls into ``self.u`` before ``replay()``."""

    def __init__(self, plan: Plan, u, psi0, psif):
        torch = _torch()
        self.plan = plan
        self.u = u.to(torch.float64).contiguous().clone()
        self.psi0 = psi0.to(torch.complex128).contiguous().clone()
        self.psif = psif.to(torch.complex128).contiguous().clone()
        self.ws = plan.workspace()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            _run(plan, self.u.reshape(-1), self.psi0, self.psif, self.ws, False)  # warm-up outside capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=side):
            self.out, self.grad = _run(plan, self.u.reshape(-1), self.psi0, self.psif, self.ws, False)

    def replay(self):
        """Run the captured step; returns (out, grad) shaped as fidelity_grad (one problem) or
        fidelity_grad_batched (out[P, 8] and the flat concatenated gradient) would."""
        self.graph.replay()
        if self.plan.P == 1:
            return self.out[0], self.grad.view(self.plan.N, self.plan.K)
        return self.out, self.grad


def _autograd_function():
    torch = _torch()

    class GrapeFidelity(torch.autograd.Function):
        """F(u) with the library's exact adjoint gradient (segment recompute inside the plan):
        the forward pass computes F and dF/du in one call and the backward pass scales the
        stored gradient.  (GrapeFidelity.apply evaluates the objective alone, without this
        Function, when no gradient can be asked for.)"""

        @staticmethod
        def forward(ctx, u, plan, psi0, psif):
            out, grad = fidelity_grad(plan, u.detach(), psi0, psif)
            ctx.save_for_backward(grad)
            return out[0].clone()

        @staticmethod
        def backward(ctx, gF):
            (grad,) = ctx.saved_tensors
            return gF * grad, None, None, None

    return GrapeFidelity


class _Lazy:
    _fn = None

    def apply(self, u, plan, psi0, psif):
        """F(u) as a 0-d tensor; differentiable in u through the library's exact gradient.
        With grad mode off or u not requiring a gradient, only the objective is evaluated
        (qoc_fidelity: no backward sweep, no gradient)."""
        torch = _torch()
        if not (torch.is_grad_enabled() and u.requires_grad):
            return fidelity(plan, u.detach(), psi0, psif)[0].clone()
        if _Lazy._fn is None:
            _Lazy._fn = _autograd_function()
        return _Lazy._fn.apply(u, plan, psi0, psif)


GrapeFidelity = _Lazy()
