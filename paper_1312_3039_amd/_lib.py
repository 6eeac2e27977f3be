"""ctypes declarations for ``libhsd.so`` (the C ABI in include/hsd.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsd.so")

OK = 0
ERR_ARG, ERR_CONE, ERR_NONFINITE, ERR_WORKSPACE, ERR_HIP, ERR_STATE, ERR_ABORTED = (
    -1, -2, -3, -4, -5, -6, -7)
SOLVED, MAX_ITERS, INFEASIBLE, UNBOUNDED, INDETERMINATE = 1, 2, 3, 4, 5
STATUS_NAMES = {SOLVED: "solved", MAX_ITERS: "max_iters", INFEASIBLE: "infeasible",
                UNBOUNDED: "unbounded", INDETERMINATE: "indeterminate"}


class HsdCone(Structure):
    _fields_ = [("f", c_int64), ("l", c_int64), ("q", POINTER(c_int32)), ("nq", c_int32),
                ("s", POINTER(c_int32)), ("ns", c_int32), ("ep", c_int64), ("ed", c_int64),
                ("p", POINTER(c_double)), ("np", c_int32)]


class HsdCsr(Structure):
    _fields_ = [("m", c_int32), ("n", c_int32), ("nnz", c_int64), ("row_ptr", c_void_p),
                ("col_idx", c_void_p), ("val", c_void_p)]


class HsdSettings(Structure):
    _fields_ = [("eps_pri", c_double), ("eps_dual", c_double), ("eps_gap", c_double),
                ("eps_unbdd", c_double), ("eps_infeas", c_double), ("alpha", c_double),
                ("cg_zeta_pow", c_double), ("cg_tight_tol", c_double),
                ("cg_max_iters", c_int32), ("max_iters", c_int32), ("check_every", c_int32),
                ("scale", c_int32), ("precision", c_int32), ("team_blocks", c_int32),
                ("block_threads", c_int32), ("lanes_a", c_int32), ("lanes_at", c_int32),
                ("lanes_soc", c_int32), ("lds_matrix", c_int32), ("slab_cols", c_int32),
                ("batch_vectors", c_int32), ("linsys", c_int32),
                ("batch_matrix", c_int32)]


class HsdInfo(Structure):
    _fields_ = [("status", c_int32), ("iters", c_int32), ("res_pri", c_double),
                ("res_dual", c_double), ("gap", c_double), ("pobj", c_double),
                ("dobj", c_double), ("obj", c_double), ("tau", c_double), ("kappa", c_double),
                ("cg_iters", c_int64), ("spmv_count", c_int64), ("setup_ms", c_double),
                ("solve_ms", c_double), ("kernel_ms", c_double), ("res_infeas", c_double),
                ("res_unbdd", c_double)]

    def to_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["status_name"] = STATUS_NAMES.get(self.status, "unknown")
        return d


class HsdLaunch(Structure):
    _fields_ = [("team_blocks", c_int32), ("block_threads", c_int32), ("lanes_a", c_int32),
                ("lanes_at", c_int32), ("lanes_soc", c_int32), ("slabs_a", c_int32),
                ("slabs_at", c_int32), ("lds_matrix", c_int32), ("row_stage", c_int32),
                ("col_stage", c_int32), ("long_rows", c_int32), ("max_row_a", c_int32),
                ("max_row_at", c_int32), ("lds_bytes", c_int64), ("vectors_lds", c_int32)]

    def to_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes); every function declared in include/hsd.h
SIGNATURES = {
    "hsd_version": (c_char_p, []),
    "hsd_last_error": (c_char_p, []),
    "hsd_default_settings": (None, [POINTER(HsdSettings)]),
    "hsd_workspace_bytes": (c_int32, [POINTER(HsdCsr), POINTER(HsdCone), POINTER(HsdSettings),
                                      POINTER(c_size_t)]),
    "hsd_setup": (c_int32, [POINTER(HsdCsr), c_void_p, c_void_p, POINTER(HsdCone),
                            POINTER(HsdSettings), c_void_p, c_size_t, c_void_p,
                            POINTER(c_void_p)]),
    "hsd_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(HsdInfo)]),
    "hsd_warm_start": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hsd_start_from_q": (c_int32, [c_void_p, c_void_p]),
    "hsd_iterate": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "hsd_get_scaling": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(c_double),
                                  POINTER(c_double)]),
    "hsd_get_launch": (c_int32, [c_void_p, POINTER(HsdLaunch)]),
    "hsd_finish": (None, [c_void_p]),
    "hsd_update_b": (c_int32, [c_void_p, c_void_p]),
    "hsd_update_bc": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "hsd_get_state": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                POINTER(c_int32)]),
    "hsd_set_state": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32]),
    "hsd_update_settings": (c_int32, [c_void_p, POINTER(HsdSettings)]),
    "hsd_project_cone": (c_int32, [POINTER(HsdCone), c_int32, c_void_p, c_void_p, c_int32,
                                   c_void_p]),
    "hsd_project_cone_noalloc": (c_int32, [POINTER(HsdCone), c_int32, c_void_p, c_void_p, c_int32,
                                           c_void_p]),
    "hsd_batch_workspace_bytes": (c_int32, [c_int32, POINTER(HsdCsr), POINTER(c_int64),
                                            POINTER(c_int64), POINTER(HsdCone),
                                            POINTER(HsdSettings), POINTER(c_size_t)]),
    "hsd_batch_setup": (c_int32, [c_int32, POINTER(HsdCsr), POINTER(c_int64), POINTER(c_int64),
                                  c_void_p, c_void_p, POINTER(HsdCone), POINTER(HsdSettings),
                                  c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "hsd_batch_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(HsdInfo)]),
    "hsd_batch_get_state": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "hsd_batch_get_launch": (c_int32, [c_void_p, POINTER(HsdLaunch)]),
    "hsd_batch_finish": (None, [c_void_p]),
    "hsd_mlp_workspace_bytes": (c_int32, [c_int32, c_int32, c_int32, c_int32, POINTER(c_size_t)]),
    "hsd_mlp_create": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p, c_size_t, c_void_p,
                                 POINTER(c_void_p)]),
    "hsd_mlp_param_count": (c_int64, [c_void_p]),
    "hsd_mlp_set_params": (c_int32, [c_void_p, c_void_p]),
    "hsd_mlp_get_params": (c_int32, [c_void_p, c_void_p]),
    "hsd_mlp_forward": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "hsd_mlp_gradients": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "hsd_mlp_train_step": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_float, c_void_p]),
    "hsd_mlp_destroy": (None, [c_void_p]),
}

_LIB = None


class HsdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hsd error {code}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    """Load libhsd.so (once).  Raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1312_3039_amd.build` "
            "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def check(code: int) -> None:
    if code != OK:
        msg = load().hsd_last_error()
        raise HsdError(code, msg.decode() if msg else "")


def make_cone(cone) -> tuple:
    """Cone description (dict or object with f, l, q, s, ep, ed and
    optionally p) -> HsdCone plus the ctypes arrays it points to (kept alive
    by the caller)."""
    if isinstance(cone, dict):
        get = lambda k: cone.get(k, [] if k == "p" else 0)  # noqa: E731
    else:
        get = lambda k: getattr(cone, k, [] if k == "p" else 0)  # noqa: E731
    q = [int(v) for v in get("q")]
    s = [int(v) for v in get("s")]
    p = [float(v) for v in get("p")]
    qa = (c_int32 * max(1, len(q)))(*q)
    sa = (c_int32 * max(1, len(s)))(*s)
    pa = (c_double * max(1, len(p)))(*p)
    K = HsdCone(f=int(get("f")), l=int(get("l")), q=qa, nq=len(q), s=sa, ns=len(s),
                ep=int(get("ep")), ed=int(get("ed")), p=pa, np=len(p))
    return K, (qa, sa, pa)
