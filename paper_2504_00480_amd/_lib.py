"""ctypes binding of libnfftgp.so: argument marshalling only.

The shared library is loaded after ``torch`` so that both use the same HIP
runtime; every computation runs in the library's HIP kernels.  There is no
fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnfftgp.so")

OK = 0
STATUS = {0: "NFFTGP_OK", -1: "NFFTGP_E_ARG", -2: "NFFTGP_E_DIM", -3: "NFFTGP_E_BOX",
          -4: "NFFTGP_E_HIP", -5: "NFFTGP_E_NOMEM", -6: "NFFTGP_E_NOTPD", -7: "NFFTGP_E_NOCONV",
          -8: "NFFTGP_E_STATE"}
E_NOTPD = -6
E_NOCONV = -7
MAX_CG_HISTORY = 4096   # NFFTGP_MAX_CG_HISTORY

# every symbol declared in include/nfftgp.h
SYMBOLS = ["nfftgp_plan_create", "nfftgp_plan_create_scaled", "nfftgp_set_hyper", "nfftgp_apply", "nfftgp_cg", "nfftgp_col_dots",
           "nfftgp_slq_logquad", "nfftgp_get_window_info", "nfftgp_get_workspace_bytes",
           "nfftgp_plan_destroy", "nfftgp_last_error", "nfftgp_profile", "nfftgp_profile_read",
           "nfftgp_autotune", "nfftgp_col_dots_noalloc", "nfftgp_precond_attach", "nfftgp_precond_info",
           "nfftgp_precond_landmarks", "nfftgp_precond_apply", "nfftgp_precond_dquad", "nfftgp_pcg",
           "nfftgp_describe"]
PROF_NAMES = ["fill", "spread", "fold", "fft_fwd", "diag", "fft_inv", "interp", "assemble", "coef", "cg",
              "gather", "precond"]
PC_MINV, PC_FINVT, PC_F = 0, 1, 2


class NfftgpError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libnfftgp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python paper_2504_00480_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.nfftgp_plan_create.argtypes = [ctypes.POINTER(P), P, i64, i32, i64, i32, P, P, P, P, i32,
                                       ctypes.c_int, i32, i32, P]
    lib.nfftgp_plan_create.restype = ctypes.c_int
    lib.nfftgp_plan_create_scaled.argtypes = [ctypes.POINTER(P), P, i64, i32, i64, i32, P, P, P, P, i32,
                                              ctypes.c_int, P, P, i32, P]
    lib.nfftgp_plan_create_scaled.restype = ctypes.c_int
    lib.nfftgp_set_hyper.argtypes = [P, f64, P, f64]
    lib.nfftgp_set_hyper.restype = ctypes.c_int
    lib.nfftgp_apply.argtypes = [P, P, i64, i32, P, P, P, P]
    lib.nfftgp_apply.restype = ctypes.c_int
    lib.nfftgp_cg.argtypes = [P, P, i32, P, f64, i32, i32, P, P, P]
    lib.nfftgp_cg.restype = ctypes.c_int
    lib.nfftgp_col_dots.argtypes = [P, P, i64, P, i64, i64, i32, P]
    lib.nfftgp_col_dots.restype = ctypes.c_int
    lib.nfftgp_col_dots_noalloc.argtypes = [ctypes.c_int, P, i64, P, i64, i64, i32, P, P]
    lib.nfftgp_col_dots_noalloc.restype = ctypes.c_int
    lib.nfftgp_slq_logquad.argtypes = [P, P, i32, i32, P, P]
    lib.nfftgp_slq_logquad.restype = ctypes.c_int
    lib.nfftgp_get_window_info.argtypes = [P, i32, P, P, P, P, P, P]
    lib.nfftgp_get_window_info.restype = ctypes.c_int
    lib.nfftgp_get_workspace_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.nfftgp_get_workspace_bytes.restype = ctypes.c_int
    lib.nfftgp_describe.argtypes = [P, i32, ctypes.c_char_p, ctypes.c_int64]
    lib.nfftgp_describe.restype = ctypes.c_int
    lib.nfftgp_plan_destroy.argtypes = [P]
    lib.nfftgp_plan_destroy.restype = None
    lib.nfftgp_profile.argtypes = [P, i32]
    lib.nfftgp_profile.restype = ctypes.c_int
    lib.nfftgp_profile_read.argtypes = [P, P, P]
    lib.nfftgp_profile_read.restype = ctypes.c_int
    lib.nfftgp_autotune.argtypes = [P, i32, i32, i32, ctypes.c_char_p, i64]
    lib.nfftgp_autotune.restype = ctypes.c_int
    lib.nfftgp_precond_attach.argtypes = [P, P, i64, i32, i32, i32]
    lib.nfftgp_precond_info.argtypes = [P, P, P, P, P]
    lib.nfftgp_precond_landmarks.argtypes = [P, P]
    lib.nfftgp_precond_apply.argtypes = [P, i32, P, i32, P]
    lib.nfftgp_precond_dquad.argtypes = [P, P, i32, P]
    lib.nfftgp_pcg.argtypes = [P, P, i32, P, f64, i32, i32, P, P, P]
    for fn in ("nfftgp_precond_attach", "nfftgp_precond_info", "nfftgp_precond_landmarks", "nfftgp_precond_apply",
               "nfftgp_precond_dquad", "nfftgp_pcg"):
        getattr(lib, fn).restype = ctypes.c_int
    lib.nfftgp_last_error.argtypes = []
    lib.nfftgp_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int, where: str):
    if status != OK:
        msg = load().nfftgp_last_error().decode(errors="replace")
        raise NfftgpError(status, where, msg)
