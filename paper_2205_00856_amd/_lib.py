"""ctypes binding of libcntri.so (the C ABI in include/cntri.h).

Argument marshalling only: every step of the solve runs in the HIP kernels of the library.
There is no CPU fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcntri.so")

CN_OK = 0
CN_NUMERICAL_BREAKDOWN = 1
CN_ERR_INVALID_ARG = -1
CN_ERR_UNSUPPORTED = -2
CN_ERR_NO_MEMORY = -3
CN_ERR_HIP = -4
CN_ERR_NOT_RESERVED = -5
CN_ERR_SCRATCH_TOO_SMALL = -6
CN_ERR_WAIT_TIMEOUT = -7


class CnLayout(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("batch", ctypes.c_int64),
        ("elem_stride", ctypes.c_int64),
        ("batch_stride", ctypes.c_int64),
        ("offsets", ctypes.POINTER(ctypes.c_int64)),
        ("partition", ctypes.c_int32),
        ("rows_per_thread", ctypes.c_int32),
        ("shared_coefficients", ctypes.c_int32),
        ("levels", ctypes.c_int32),
    ]


class CnOperator(ctypes.Structure):
    _fields_ = [
        ("V", ctypes.c_void_p),
        ("v_scale", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("dx_per_system", ctypes.c_void_p),
        ("dt", ctypes.c_double),
        ("xgrid", ctypes.c_void_p),
        ("absorb", ctypes.c_void_p),
    ]


class CnRadial(ctypes.Structure):
    _fields_ = [
        ("nr", ctypes.c_int64),
        ("l0", ctypes.c_int64),
        ("nl", ctypes.c_int64),
        ("V", ctypes.c_void_p),
        ("dr", ctypes.c_double),
        ("dt", ctypes.c_double),
    ]


class CnError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None


def lib():
    """Load libcntri.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2205_00856_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    H = ctypes.c_void_p
    LP = ctypes.POINTER(CnLayout)
    OP = ctypes.POINTER(CnOperator)
    i64 = ctypes.c_int64
    d = ctypes.c_double
    sig = {
        "cn_check_layout": ([LP], ctypes.c_int),
        "cn_create": ([ctypes.POINTER(H), ctypes.c_int], ctypes.c_int),
        "cn_destroy": ([H], ctypes.c_int),
        "cn_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "cn_reserve": ([H, LP], ctypes.c_int),
        "cn_tridiag_solve": ([H, LP, P, P, P, P, P, P], ctypes.c_int),
        "cn_tridiag_solve_noalloc": ([H, LP, P, P, P, P, P, P], ctypes.c_int),
        "cn_tridiag_solve_adjoint": ([H, LP, P, P, P, P, P, P, P, P, P, P], ctypes.c_int),
        "cn_assemble": ([H, LP, OP, d, P, P, P, P], ctypes.c_int),
        "cn_rhs": ([H, LP, OP, d, P, P, P], ctypes.c_int),
        "cn_step": ([H, LP, OP, d, P, P, P], ctypes.c_int),
        "cn_propagate": ([H, LP, OP, i64, P, P, P, i64, P], ctypes.c_int),
        "cn_propagate_resident": ([H, LP, OP, i64, P, P, P, i64, P], ctypes.c_int),
        "cn_step_adjoint": ([H, LP, OP, d, P, P, P, P, P, P, P], ctypes.c_int),
        "cn_get_status": ([H, P], ctypes.c_int),
        "cn_version": ([], ctypes.c_char_p),
        "cn_describe_plan": ([H, LP, ctypes.c_int, ctypes.c_char_p, i64], ctypes.c_int),
        "cn_propagate_adjoint": ([H, LP, OP, i64, P, P, i64, P, P, P, P, P], ctypes.c_int),
        "cn_propagate_adjoint_reconstruct": ([H, LP, OP, i64, P, P, i64, P, P, P, P, P],
                                             ctypes.c_int),
        "cn_autotune": ([H, LP, ctypes.c_int, OP, d, P, P, P, P, P, ctypes.c_char_p, i64, P],
                        ctypes.c_int),
        "cn_handle_info": ([H, ctypes.POINTER(i64), ctypes.POINTER(i64),
                            ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "cn_profile": ([H, ctypes.c_int], ctypes.c_int),
        "cn_tune_cache": ([H, ctypes.c_char_p], ctypes.c_int),
        "cn_radial_step": ([H, ctypes.POINTER(CnRadial), d, P, P, P], ctypes.c_int),
        "cn_profile_report": ([H, ctypes.c_char_p, i64], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


EXPORTED = ["cn_check_layout", "cn_create", "cn_destroy", "cn_status_string", "cn_reserve", "cn_tridiag_solve",
            "cn_tridiag_solve_adjoint", "cn_assemble", "cn_rhs", "cn_step", "cn_propagate",
            "cn_propagate_resident", "cn_step_adjoint", "cn_get_status", "cn_version", "cn_describe_plan", "cn_autotune",
            "cn_propagate_adjoint", "cn_propagate_adjoint_reconstruct", "cn_handle_info", "cn_tridiag_solve_noalloc", "cn_profile",
            "cn_profile_report", "cn_tune_cache", "cn_radial_step"]


def status_string(st: int) -> str:
    try:
        return lib().cn_status_string(st).decode()
    except Exception:  # noqa: BLE001 - only used to format an error message
        return str(st)


def check(st: int, what: str) -> int:
    if st < 0:
        raise CnError(st, what)
    return st
