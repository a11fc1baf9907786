"""ctypes declarations of the libcpamg C ABI (include/cpamg.h).

Loading fails loudly: there is no fallback implementation of any call.
"""
from __future__ import annotations

import ctypes
import os

CP_MAX_ORDER = 8
CP_MAX_RANK = 32
CP_MAX_RESTARTS = 8
CP_NOALLOC_SCRATCH_BYTES = 32 << 20

CP_OK = 0
CP_ERR_INVALID = -1
CP_ERR_SHAPE = -2
CP_ERR_NOT_SPD = -3
CP_ERR_NONFINITE = -4
CP_ERR_HIP = -5
CP_ERR_NOMEM = -6
CP_ERR_UNSUPPORTED = -7

CP_FP64 = 0
CP_MIXED = 1
CP_SOLVE_CHOL = 0
CP_SOLVE_GS = 1

PROF_CLASSES = ["mttkrp_mode0_f64", "mttkrp_mode1_f64", "mttkrp_modeN_f64",
                "mttkrp_mode0_f32", "mttkrp_mode1_f32", "mttkrp_modeN_f32",
                "update", "epilogue_other", "gamma_prep", "normalize", "gram", "other"]

CP_OPT_DIMTREE = 1
CP_OPT_GRAPHS = 2
CP_OPT_SMALL_LEVELS = 3

CP_FLAG_PINV_FALLBACK = 1
CP_FLAG_NOT_SPD = 2
CP_FLAG_NONFINITE = 4

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcpamg.so")

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_vp = ctypes.c_void_p


class CpTensor(ctypes.Structure):
    _fields_ = [("order", c_i32), ("dims", c_i64 * CP_MAX_ORDER), ("z64", c_vp),
                ("z32", c_vp), ("norm2", c_vp), ("nnz", c_i64), ("idx", c_vp), ("vals", c_vp),
                ("rowptr", c_vp * CP_MAX_ORDER), ("perm", c_vp * CP_MAX_ORDER)]


class CpFactors(ctypes.Structure):
    _fields_ = [("rank", c_i32), ("a", c_vp * CP_MAX_ORDER), ("a32", c_vp * CP_MAX_ORDER)]


class CpLevel(ctypes.Structure):
    _fields_ = [("z", CpTensor), ("phat", c_vp * CP_MAX_ORDER)]


class CpFasParams(ctypes.Structure):
    _fields_ = [("nu1", c_i32), ("nu2", c_i32), ("nuc", c_i32), ("gs_iters", c_i32),
                ("ic_rule", c_i32)]


class CpBatchProblem(ctypes.Structure):
    _fields_ = [("z", CpTensor), ("a", CpFactors)]


class CpBatchParams(ctypes.Structure):
    _fields_ = [("restarts", c_i32), ("prec", c_i32), ("window32", c_i32), ("tol32", ctypes.c_double),
                ("tol64", ctypes.c_double), ("max_sweeps", c_i32), ("chunk", c_i32), ("wg_kib", c_i32)]


# name -> (argtypes)
SIGNATURES = {
    "cp_ctx_create": [ctypes.POINTER(c_vp), c_vp],
    "cp_ctx_destroy": [c_vp],
    "cp_set_stream": [c_vp, c_vp],
    "cp_set_option": [c_vp, c_i32, c_i32],
    "cp_get_status": [c_vp, ctypes.POINTER(c_i32)],
    "cp_cast_f32": [c_vp, c_vp, c_vp, c_i64],
    "cp_norm2": [c_vp, ctypes.POINTER(CpTensor), c_vp],
    "cp_sparse_index": [c_vp, c_i32, ctypes.POINTER(c_i64), c_i64, c_vp, c_vp, c_vp],
    "cp_mttkrp": [c_vp, ctypes.POINTER(CpTensor), ctypes.POINTER(CpFactors), c_i32, c_vp, c_i32],
    "cp_mttkrp_noalloc": [c_vp, ctypes.POINTER(CpTensor), ctypes.POINTER(CpFactors), c_i32, c_vp,
                          c_i32],
    "cp_als_sweep": [c_vp, ctypes.POINTER(CpTensor), ctypes.POINTER(CpFactors),
                     ctypes.POINTER(CpFactors), c_i32, c_i32, c_i32, c_i32, c_i32, c_vp],
    "cp_objective": [c_vp, ctypes.POINTER(CpTensor), ctypes.POINTER(CpFactors), c_i32, c_vp,
                     c_vp, c_i32],
    "cp_restrict": [c_vp, ctypes.POINTER(CpTensor), c_vp * CP_MAX_ORDER, ctypes.POINTER(CpTensor),
                    c_i32],
    "cp_restrict_factored": [c_vp, ctypes.POINTER(CpTensor), c_vp * CP_MAX_ORDER, ctypes.POINTER(CpTensor),
                             c_i32],
    "cp_prolong": [c_vp, c_i64, c_i64, c_i32, c_vp, c_vp, c_vp, c_vp],
    "cp_restrict_factor": [c_vp, c_i64, c_i64, c_i32, c_vp, c_vp, c_vp],
    "cp_transfer_build": [c_vp, c_i64, c_vp, c_vp],
    "cp_interp_weights": [c_vp, ctypes.POINTER(CpTensor), ctypes.POINTER(CpFactors), c_i32, c_i32, c_i32,
                          c_vp],
    "cp_fas_vcycle": [c_vp, ctypes.POINTER(CpLevel), c_i32, ctypes.POINTER(CpFactors),
                      ctypes.POINTER(CpFasParams), c_i32],
    "cp_sort": [c_vp, ctypes.POINTER(c_i64), c_i32, ctypes.POINTER(CpFactors)],
    "cp_profile_enable": [c_vp, c_i32],
    "cp_autotune": [c_vp, ctypes.POINTER(CpTensor), ctypes.POINTER(CpFactors), c_i32, c_i32],
    "cp_plans_import": [c_vp, ctypes.c_char_p],
    "cp_time_mttkrp": [c_vp, ctypes.POINTER(CpTensor), ctypes.POINTER(CpFactors), c_i32, c_i32,
                       c_i32, ctypes.POINTER(ctypes.c_double)],
    "cp_profile_read": [c_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_i32)],
    "cp_als_batched": [c_vp, ctypes.POINTER(CpBatchProblem), c_i32, ctypes.POINTER(CpBatchParams),
                       c_vp, c_vp],
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libcpamg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libcpamg.so not found at {path}: build it first "
            "(python -m paper_1111_6091_amd.build); there is no fallback path")
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c_i32
    lib.cp_last_error.argtypes = [c_vp]
    lib.cp_last_error.restype = ctypes.c_char_p
    lib.cp_plans_export.argtypes = [c_vp]
    lib.cp_plans_export.restype = ctypes.c_char_p
    _lib = lib
    return lib


def exported_names():
    return list(SIGNATURES) + ["cp_last_error", "cp_plans_export"]
