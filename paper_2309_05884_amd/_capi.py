"""ctypes declarations of include/qoc.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# QOC_LIBRARY may name another build of the same library (same ABI), e.g. a tuned variant
LIB_PATH = os.environ.get("QOC_LIBRARY") or os.path.join(HERE, "libqoc_gfx950.so")

QOC_OK = 0
STATUS = {0: "QOC_OK", 1: "QOC_ERR_INVALID_ARG", 2: "QOC_ERR_SYMMETRY", 3: "QOC_ERR_UNSUPPORTED",
          4: "QOC_ERR_OUT_OF_MEMORY", 5: "QOC_ERR_DEVICE", 6: "QOC_ERR_NUMERIC"}
STATUS_CODE = {v: k for k, v in STATUS.items()}
GROUPS = {"dihedral": 0, "cyclic": 1, "symmetric": 2}
PRECISIONS = {"c128": 0, "c64": 1}
TERM_KINDS = {"one_body": 0, "ring_pair": 1, "all_pairs": 2, "pauli": 3}
SITES = {"all": 0, "even": 1, "odd": 2}


class QocTerm(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("distance", ctypes.c_int32), ("sites", ctypes.c_int32),
                ("staggered", ctypes.c_int32), ("coeff", ctypes.c_double), ("op_a", ctypes.c_char),
                ("op_b", ctypes.c_char), ("pad_", ctypes.c_char * 6), ("x_mask", ctypes.c_uint64),
                ("z_mask", ctypes.c_uint64)]


class QocLbfgsOptions(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("memory", ctypes.c_int), ("step0", ctypes.c_double),
                ("c1", ctypes.c_double), ("max_backtrack", ctypes.c_int), ("f_target", ctypes.c_double),
                ("gtol", ctypes.c_double)]


class QocLbfgsResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("evaluations", ctypes.c_int), ("reason", ctypes.c_int),
                ("F", ctypes.c_double)]


OPT_REASONS = {0: "target", 1: "gtol", 2: "max_iter", 3: "line_search_failed"}


class QocError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        self.code = STATUS.get(status, str(status))
        super().__init__(f"{self.code}: {detail}")


_lib = None

vp = ctypes.c_void_p
PROTOTYPES = {
    "qoc_build_basis": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(vp)]),
    "qoc_basis_free": (None, [vp]),
    "qoc_basis_blocks": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32), ctypes.c_int]),
    "qoc_basis_reps": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64)]),
    "qoc_state_to_blocks": (ctypes.c_int, [vp, vp, vp, vp]),
    "qoc_state_from_blocks": (ctypes.c_int, [vp, vp, vp, vp]),
    "qoc_project": (ctypes.c_int, [vp, ctypes.POINTER(QocTerm), ctypes.c_int, ctypes.POINTER(QocTerm),
                                   ctypes.POINTER(ctypes.c_int), ctypes.c_int, vp, ctypes.POINTER(vp)]),
    "qoc_system_free": (None, [vp]),
    "qoc_check_symmetry": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(QocTerm),
                                          ctypes.c_int]),
    "qoc_system_block": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, vp]),
    "qoc_plan_create": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_size_t, ctypes.POINTER(vp)]),
    "qoc_plan_create_batched": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                               ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_double,
                                               ctypes.c_size_t, ctypes.POINTER(vp)]),
    "qoc_plan_create_blocks": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_size_t,
                                              ctypes.POINTER(vp)]),
    "qoc_plan_free": (None, [vp]),
    "qoc_plan_workspace_size": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_size_t)]),
    "qoc_plan_info": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]),
    "qoc_propagate": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_size_t, vp]),
    "qoc_fidelity_grad": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
    "qoc_fidelity": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
    "qoc_fidelity_grad_noalloc": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
    "qoc_plan_read_state": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp,
                                           vp]),
    "qoc_plan_set_sweep_mode": (ctypes.c_int, [vp, ctypes.c_int]),
    "qoc_plan_set_generator_split": (ctypes.c_int, [vp, ctypes.c_int]),
    "qoc_measure_mfma_peak": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double), vp]),
    "qoc_plan_groups": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.c_int]),
    "qoc_set_progress": (ctypes.c_int, [ctypes.c_int]),
    "qoc_set_products_policy": (ctypes.c_int, [ctypes.c_int]),
    "qoc_profile_begin": (ctypes.c_int, [ctypes.c_int]),
    "qoc_profile_end": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), ctypes.c_int]),
    "qoc_plan_slice_stats": (ctypes.c_int, [vp, vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_double), vp]),
    "qoc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "qoc_last_error": (ctypes.c_char_p, []),
    "qoc_version": (ctypes.c_int, []),
    "qoc_plan_set_variant": (ctypes.c_int, [vp, ctypes.c_int]),
    "qoc_variant_name": (ctypes.c_char_p, [ctypes.c_int, ctypes.c_int]),
    "qoc_plan_autotune": (ctypes.c_int, [vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_double)]),
    "qoc_lts_workspace_size": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "qoc_lts_apply": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, vp, ctypes.c_int, ctypes.c_double,
                                     vp, ctypes.c_int, vp, vp, ctypes.c_size_t, vp]),
    "qoc_lts_grad_workspace_size": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "qoc_lts_fidelity_grad": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, vp, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_int, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
    "qoc_gate_propagate": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_size_t, vp]),
    "qoc_gate_fidelity": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
    "qoc_optimize_lts_workspace_size": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                       ctypes.POINTER(ctypes.c_size_t)]),
    "qoc_optimize_lbfgs_lts": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_double, ctypes.POINTER(QocLbfgsOptions), vp, vp, vp, vp,
                                              ctypes.c_size_t, vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                              ctypes.POINTER(QocLbfgsResult)]),
    "qoc_optimize_workspace_size": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "qoc_optimize_lbfgs": (ctypes.c_int, [vp, ctypes.POINTER(QocLbfgsOptions), vp, vp, vp, vp, ctypes.c_size_t, vp,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                          ctypes.POINTER(QocLbfgsResult)]),
}


def lib():
    """The loaded HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2309_05884_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != QOC_OK:
        detail = lib().qoc_last_error().decode(errors="replace")
        raise QocError(status, detail)


def make_terms(terms):
    """Convert term descriptors (dicts, see qoc_workloads) into a QocTerm array."""
    arr = (QocTerm * max(1, len(terms)))()
    for i, t in enumerate(terms):
        q = arr[i]
        q.kind = TERM_KINDS[t["kind"]]
        q.coeff = float(t["coeff"])
        if t["kind"] == "one_body":
            q.op_a = t["op"].encode()
            q.sites = SITES[t.get("sites", "all")]
            q.staggered = 1 if t.get("stagger") else 0
        elif t["kind"] in ("ring_pair", "all_pairs"):
            q.op_a = t["op"][0].encode()
            q.op_b = t["op"][1].encode()
            q.distance = int(t.get("distance", 1))
        elif t["kind"] == "pauli":
            s = t["string"]
            n = len(s)
            xm = zm = 0
            for idx, ch in enumerate(s):
                p = n - (idx + 1)  # qubit idx+1 sits at bit position n - q
                ch = ch.upper()
                if ch in "XY":
                    xm |= 1 << p
                if ch in "ZY":
                    zm |= 1 << p
            q.x_mask = xm
            q.z_mask = zm
    return arr
