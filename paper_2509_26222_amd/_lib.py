"""ctypes declarations of librbf.so (see include/rbf.h).

The library is loaded from this package directory only; there is no
fallback. Importing this module raises if librbf.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librbf.so")

RBF_OK = 0
STATUS_NAMES = {
    0: "RBF_OK", 1: "RBF_E_INVALID_ARG", 2: "RBF_E_NOMEM", 3: "RBF_E_NOT_SPD",
    4: "RBF_E_NONFINITE", 5: "RBF_E_NO_CONVERGE", 6: "RBF_E_CAPACITY",
    7: "RBF_E_HIP",
}
F64, F32, BF16 = 0, 1, 2
SELECT_RADIUS, SELECT_VOXEL = 0, 1
RBF_TILE_AUTO, RBF_TILE_128, RBF_TILE_SUB = 0, 1, 2


class Params(C.Structure):
    _fields_ = [("sigma", C.c_double), ("cutoff", C.c_double),
                ("sigma_eps", C.c_double), ("lambda_", C.c_double),
                ("R", C.c_double)]


vp = C.c_void_p
i64 = C.c_int64
i32 = C.c_int32
dbl = C.c_double
pp = C.POINTER(Params)


class Patch(C.Structure):
    """rbf_patch (include/rbf.h)."""
    _fields_ = [("grid", vp), ("w", vp), ("P", vp), ("ldp", i64), ("xy", vp), ("z", vp),
                ("M", i64), ("pts", vp), ("Q", i64), ("pose", dbl * 12), ("f", vp),
                ("grad", vp), ("resid", vp), ("jac", vp), ("batch", i64)]

class CSR(C.Structure):
    """rbf_csr (include/rbf.h)."""
    _fields_ = [("n", i64), ("nnz", i64), ("rowptr", vp), ("colidx", vp), ("vals", vp)]


ASSEMBLE_PHI, ASSEMBLE_GRAM = 1, 2

# name -> (restype, argtypes)
SIGNATURES = {
    "rbf_ctx_create": (C.c_int, [C.POINTER(vp), C.c_int, vp]),
    "rbf_ctx_destroy": (C.c_int, [vp]),
    "rbf_ctx_set_stream": (C.c_int, [vp, vp]),
    "rbf_ctx_set_update_streams": (C.c_int, [vp, i32]),
    "rbf_ctx_set_update_joseph": (C.c_int, [vp, i32]),
    "rbf_sync_status": (C.c_int, [vp]),
    "rbf_last_error_index": (i64, [vp]),
    "rbf_last_error": (C.c_char_p, [vp]),
    "rbf_status_string": (C.c_char_p, [C.c_int]),
    "rbf_select_centers": (C.c_int, [vp, vp, i64, C.POINTER(dbl), dbl, dbl, i32,
                                     i32, vp, i64, C.POINTER(i64)]),
    "rbf_select_centers_grow": (C.c_int, [vp, vp, i64, C.POINTER(dbl), dbl, dbl, i32, i32,
                                          vp, vp, i64, C.POINTER(i64)]),
    "rbf_state_grow": (C.c_int, [vp, pp, vp, vp, i64, i64, i64]),
    "rbf_grid_create": (C.c_int, [vp, pp, vp, i64, C.POINTER(vp)]),
    "rbf_grid_destroy": (C.c_int, [vp]),
    "rbf_bin_centers": (C.c_int, [vp, vp, i64, pp, C.POINTER(vp)]),
    "rbf_grid_set_mesh": (C.c_int, [vp, vp, dbl, dbl, dbl]),
    "rbf_grid_info": (C.c_int, [vp, C.POINTER(i64), C.POINTER(i32),
                                C.POINTER(i32), C.POINTER(i32)]),
    "rbf_sort_points": (C.c_int, [vp, vp, vp, vp, i64, vp, vp, vp]),
    "rbf_assemble_phi": (C.c_int, [vp, pp, vp, vp, i64, C.c_int, vp, vp, vp, i32]),
    "rbf_gram_pattern": (C.c_int, [vp, pp, vp, vp, vp, i64, C.POINTER(i64)]),
    "rbf_assemble_gram": (C.c_int, [vp, pp, vp, vp, vp, i64, vp, vp, vp, vp, i32]),
    "rbf_assemble": (C.c_int, [vp, pp, vp, vp, vp, i64, i32, C.c_int, vp, vp, vp, i32,
                               C.POINTER(CSR), vp, i32]),
    "rbf_update": (C.c_int, [vp, pp, vp, vp, vp, i64, vp, vp, i64, i64, C.c_int,
                             C.POINTER(i64)]),
    "rbf_update_active": (C.c_int, [vp, pp, vp, vp, vp, i64, vp, vp, i64, i64, C.c_int,
                                    vp, C.POINTER(i64), C.POINTER(i64)]),
    "rbf_solve": (C.c_int, [vp, i64, vp, vp, vp, vp, i64, vp, i64, i64, dbl, i32,
                            C.c_int, C.POINTER(dbl), C.POINTER(i32)]),
    "rbf_solve_plan_create": (C.c_int, [vp, i64, vp, vp, i32, C.POINTER(vp)]),
    "rbf_solve_plan_run": (C.c_int, [vp, vp, vp, i64, vp, i64, i64, dbl, i32, C.c_int,
                                     C.POINTER(dbl), C.POINTER(i32)]),
    "rbf_solve_plan_info": (C.c_int, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i64),
                                      C.POINTER(i32)]),
    "rbf_solve_plan_destroy": (C.c_int, [vp]),
    "rbf_solve_order_host": (C.c_int, [i64, vp, vp, i32, vp, vp, vp, i32, C.POINTER(i32)]),
    "rbf_refine": (C.c_int, [vp, i64, vp, vp, vp, vp, vp, i64, dbl, vp, dbl, i32,
                             C.POINTER(dbl), C.POINTER(i32)]),
    "rbf_eval": (C.c_int, [vp, pp, vp, vp, vp, i64, i32, C.POINTER(dbl), dbl,
                           C.c_int, vp, vp, vp, vp]),
    "rbf_eval_noalloc": (C.c_int, [vp, pp, vp, vp, vp, i64, i32, C.POINTER(dbl), dbl,
                                   C.c_int, vp, vp, vp, vp]),
    "rbf_eval_at": (C.c_int, [vp, pp, vp, vp, vp, i64, C.POINTER(dbl), vp, dbl, C.c_int, vp,
                              vp, vp, vp]),
    "rbf_eval_adjoint_at": (C.c_int, [vp, pp, vp, vp, vp, i64, C.POINTER(dbl), vp, C.c_int,
                                      vp, vp, vp, vp, vp]),
    "rbf_eval_gn": (C.c_int, [vp, pp, vp, vp, vp, i64, C.POINTER(dbl), dbl, C.c_int, vp, vp,
                              vp]),
    "rbf_eval_adjoint": (C.c_int, [vp, pp, vp, vp, vp, i64, i32, C.POINTER(dbl),
                                   C.c_int, vp, vp, vp, vp, vp]),
    "rbf_batched_plan": (C.c_int, [vp, pp, vp, i32, i32, C.c_int, C.c_int, i32, i32,
                                   i64, dbl, C.POINTER(vp)]),
    "rbf_batched_run": (C.c_int, [vp]),
    "rbf_batched_sync": (C.c_int, [vp, C.POINTER(i32)]),
    "rbf_batched_destroy": (C.c_int, [vp]),
    "rbf_profile_enable": (C.c_int, [vp, i32]),
    "rbf_profile_read": (C.c_int, [vp, i32, C.POINTER(dbl), C.POINTER(i64)]),
}
PROF_SYRK, PROF_EVAL, PROF_TRSM, PROF_CHOL, PROF_GATHER = range(5)


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_2509_26222_amd.build`"
            " (there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB
