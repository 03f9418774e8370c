"""The C ABI library on the host: it loads, exports every declared entry point, and
rejects invalid arguments before touching the device (no compute calls here)."""
import ctypes
import os
import re

import pytest

import qoc_workloads as W
from paper_2309_05884_amd import _capi as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "qoc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(qoc_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = C.lib()
    names = declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), name
        assert name in C.PROTOTYPES, f"binding lacks {name}"


def test_status_strings_and_version():
    L = C.lib()
    for s in range(7):
        assert L.qoc_status_string(s)
    assert L.qoc_version() >= 100


def test_term_struct_layout():
    assert ctypes.sizeof(C.QocTerm) == 48
    assert C.QocTerm.coeff.offset == 16 and C.QocTerm.x_mask.offset == 32


def test_optimizer_struct_layout():
    """The ctypes mirrors of qoc_lbfgs_options / qoc_lbfgs_result match the C layout
    (natural alignment on x86-64)."""
    assert ctypes.sizeof(C.QocLbfgsOptions) == 48
    assert C.QocLbfgsOptions.step0.offset == 8 and C.QocLbfgsOptions.max_backtrack.offset == 24
    assert C.QocLbfgsOptions.f_target.offset == 32 and C.QocLbfgsOptions.gtol.offset == 40
    assert ctypes.sizeof(C.QocLbfgsResult) == 24 and C.QocLbfgsResult.F.offset == 16


@pytest.mark.parametrize("n,group,stride", [(0, 0, 1), (31, 0, 1), (6, 0, 4), (6, 7, 1), (5000, 2, 1), (6, 1, 0)])
def test_build_basis_rejects_bad_arguments(n, group, stride):
    L = C.lib()
    h = ctypes.c_void_p()
    assert L.qoc_build_basis(n, group, stride, None, ctypes.byref(h)) == 1
    assert h.value is None
    assert L.qoc_last_error()


def test_null_handles_rejected():
    L = C.lib()
    nb = ctypes.c_int()
    assert L.qoc_basis_blocks(None, ctypes.byref(nb), None, None, 0) == 1
    out = ctypes.c_void_p()
    assert L.qoc_project(None, None, 0, None, None, 0, None, ctypes.byref(out)) == 1
    assert L.qoc_plan_create(None, 0, 10, 0.1, 1.0, 0, ctypes.byref(out)) == 1
    blocks = (ctypes.c_int * 1)(0)
    assert L.qoc_plan_create_blocks(None, blocks, 1, 0, 10, 0.1, 1.0, 0, ctypes.byref(out)) == 1
    assert L.qoc_fidelity_grad(None, None, None, None, None, None, None, 0, None) == 1
    assert L.qoc_propagate(None, None, None, None, 0, None) == 1
    nbytes = ctypes.c_size_t()
    assert L.qoc_optimize_workspace_size(None, 10, ctypes.byref(nbytes)) == 1
    opts = C.QocLbfgsOptions(10, 10, 0.1, 1e-4, 20, 1.0, 0.0)
    res = C.QocLbfgsResult()
    assert L.qoc_optimize_lbfgs(None, ctypes.byref(opts), None, None, None, None, 0, None, None, 0,
                                ctypes.byref(res)) == 1
    assert L.qoc_gate_propagate(None, None, None, None, 0, None) == 1
    assert L.qoc_gate_fidelity(None, None, None, None, None, 0, None) == 1
    assert L.qoc_lts_apply(4, 1.0, 1.0, None, 10, 0.1, None, 1, None, None, 0, None) == 1


def test_lts_sizes_host_only():
    """The Trotterised path keeps a column of 2^n amplitudes in LDS: n <= 13."""
    L = C.lib()
    nbytes = ctypes.c_size_t()
    assert L.qoc_lts_workspace_size(11, 100, ctypes.byref(nbytes)) == 0 and nbytes.value == 100 * 11 * 4 * 16
    assert L.qoc_lts_workspace_size(14, 100, ctypes.byref(nbytes)) == 3
    assert L.qoc_lts_workspace_size(0, 100, ctypes.byref(nbytes)) == 3
    assert L.qoc_lts_workspace_size(5, 0, ctypes.byref(nbytes)) == 1
    assert L.qoc_lts_grad_workspace_size(12, 10, 2, ctypes.byref(nbytes)) == 0 and nbytes.value == 2 * 10 * 12 * 12 * 16
    assert L.qoc_lts_grad_workspace_size(13, 10, 1, ctypes.byref(nbytes)) == 3
    assert L.qoc_lts_fidelity_grad(4, 1.0, 1.0, None, 10, 0.1, 1, None, None, None, None, None, 0, None) == 1


def test_symmetric_basis_is_host_only():
    """S_n blocks need no enumeration: sizes 2J+1 for J = n/2, n/2-1, ... (App. A)."""
    L = C.lib()
    h = ctypes.c_void_p()
    assert L.qoc_build_basis(128, 2, 1, None, ctypes.byref(h)) == 0
    nb = ctypes.c_int()
    sizes = (ctypes.c_int32 * 80)()
    copies = (ctypes.c_int32 * 80)()
    assert L.qoc_basis_blocks(h, ctypes.byref(nb), sizes, copies, 80) == 0
    assert nb.value == 65
    assert [sizes[i] for i in range(65)] == list(range(129, 0, -2))
    assert all(copies[i] == 1 for i in range(65))
    cnt = ctypes.c_int64()
    assert L.qoc_basis_reps(h, 0, None, 0, ctypes.byref(cnt)) == 3  # no enumeration for S_n
    L.qoc_basis_free(h)


def _check(n, group, stride, terms):
    arr = C.make_terms(terms)
    return C.lib().qoc_check_symmetry(n, group, stride, arr, len(terms))


def test_symmetry_check_accepts_paper_hamiltonians():
    """Sec. II A: field sums are S_n and D_n invariant; the ring coupling is D_n invariant."""
    for n in (3, 6, 12, 14):
        assert _check(n, 0, 1, W.heisenberg_ring_terms(0.9)) == 0
        assert _check(n, 0, 1, W.ising_ring_terms(1.0, 0.3)) == 0
        assert _check(n, 1, 1, W.full_coupling_terms(n, 1.0, [0.3] * (n // 2))) == 0
        assert _check(n, 2, 1, [W.one_body(1.0, "x"), W.all_pairs(0.2, "zz")]) == 0


def test_symmetry_check_rejects_broken_terms():
    stag = [W.one_body(1.0, "z", stagger=True)]
    even = [W.one_body(1.0, "x", sites="even")]
    # staggered / even-site fields break the one-site rotation but keep the two-site group
    assert _check(14, 0, 1, stag) == 2
    assert _check(14, 0, 1, even) == 2
    assert _check(14, 0, 2, stag) == 0
    assert _check(14, 0, 2, even) == 0
    # ring coupling is not S_n symmetric
    assert _check(6, 2, 1, [W.ring_pair(1.0, "zz")]) == 2
    # an xy ring pair is not reflection symmetric, but it is rotation symmetric
    assert _check(6, 0, 1, [W.ring_pair(1.0, "xy")]) == 2
    assert _check(6, 1, 1, [W.ring_pair(1.0, "xy")]) == 0
    # a single Pauli string breaks both
    assert _check(4, 1, 1, [{"kind": "pauli", "coeff": 1.0, "string": "XIII"}]) == 2


def test_symmetry_check_rejects_malformed_terms():
    assert _check(6, 0, 1, [W.one_body(float("nan"), "x")]) == 1
    assert _check(6, 0, 1, [W.one_body(1.0, "q")]) == 1
    assert _check(6, 0, 1, [W.ring_pair(1.0, "zz", 6)]) == 1


def test_gemm_variant_names_and_bad_handles():
    """Three GEMM tile variants per precision, named by precision and work-group tile;
    variant selection and autotuning reject null plans and out-of-range indices on the host."""
    L = C.lib()
    for prec, tag in ((0, "fp64"), (1, "fp32")):
        names = [L.qoc_variant_name(prec, v).decode() for v in range(3)]
        assert all(n.startswith(tag + " ") and "x" in n for n in names), names
        assert len(set(names)) == 3
        assert L.qoc_variant_name(prec, 3) == b"" and L.qoc_variant_name(prec, -1) == b""
    assert L.qoc_plan_set_variant(None, 0) == C.STATUS_CODE["QOC_ERR_INVALID_ARG"]
    assert L.qoc_plan_autotune(None, None, None, 0, None, None, None) == C.STATUS_CODE["QOC_ERR_INVALID_ARG"]
