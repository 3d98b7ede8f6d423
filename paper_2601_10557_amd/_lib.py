"""ctypes declarations of libchase_ph.so (the C ABI in include/chase_ph.h).

The library is loaded from this package directory; importing fails loudly
if it has not been built (``python -m paper_2601_10557_amd.build``).
There is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchase_ph.so")

OK, ERR_ARG, ERR_ALLOC, ERR_HIP, ERR_NOT_DEFINITE, ERR_QR, ERR_SINGULAR_QSQ, ERR_NO_CONVERGENCE, ERR_EIG = range(9)
FP64, MIXED, FP32, FP64_KREAL = 0, 1, 2, 3

STATUS_NAMES = {
    0: "OK", 1: "ERR_ARG", 2: "ERR_ALLOC", 3: "ERR_HIP", 4: "ERR_NOT_DEFINITE",
    5: "ERR_QR", 6: "ERR_SINGULAR_QSQ", 7: "ERR_NO_CONVERGENCE", 8: "ERR_EIG",
}


class Params(C.Structure):
    _fields_ = [
        ("m", C.c_int64), ("nev", C.c_int32), ("nex", C.c_int32), ("deg", C.c_int32),
        ("deg_min", C.c_int32), ("deg_max", C.c_int32), ("opt_deg", C.c_int32),
        ("max_iter", C.c_int32), ("tol", C.c_double), ("precision", C.c_int32),
        ("switch_tol", C.c_double), ("gamma", C.c_double), ("lanczos_steps", C.c_int32),
        ("lanczos_vecs", C.c_int32), ("a_conj", C.c_int32), ("rr_backup", C.c_int32),
        ("definite", C.c_int32), ("tda", C.c_int32), ("nex_auto", C.c_int32),
        ("rr_max_sweeps", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32), ("locked", C.c_int32), ("shifted_qr_used", C.c_int32),
        ("switch_iter", C.c_int32), ("mu1", C.c_double), ("mu_nevex0", C.c_double),
        ("mu_n", C.c_double), ("t_lanczos", C.c_double), ("t_filter", C.c_double),
        ("t_qr", C.c_double), ("t_rr", C.c_double), ("t_resid", C.c_double),
        ("t_total", C.c_double), ("filter_flops", C.c_double), ("rr_flops", C.c_double),
        ("filter_flops_fp32", C.c_double), ("resid_history", C.POINTER(C.c_double)),
        ("resid_history_len", C.c_int32), ("householder_qr_used", C.c_int32),
        ("backup_rr_used", C.c_int32), ("general_rr_used", C.c_int32), ("nex_used", C.c_int32),
        ("rr_sweeps_max", C.c_int32), ("qr_one_pass", C.c_int32),
    ]


EXPORTS = [
    "chase_ph_default_params", "chase_ph_create", "chase_ph_destroy", "chase_ph_last_error",
    "chase_ph_apply_h", "chase_ph_filter", "chase_ph_qr", "chase_ph_oblique_rr", "chase_ph_oblique_rr_backup",
    "chase_ph_residuals", "chase_ph_solve", "chase_ph_eigval_backward", "chase_ph_last_timing",
    "chase_ph_profile", "chase_ph_profile_read", "chase_ph_filter_refined", "chase_ph_mfma_probe",
    "chase_ph_eigval_backward_noalloc", "chase_ph_oblique_rr_general",
]

NOALLOC_MAX_NEV = 16384   # CHASE_PH_NOALLOC_MAX_NEV


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"{path} not found: build the HIP library first "
            "(python -m paper_2601_10557_amd.build); there is no fallback path")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    pd = C.POINTER(C.c_double)
    pi = C.POINTER(C.c_int32)
    lib.chase_ph_default_params.argtypes = [C.POINTER(Params)]
    lib.chase_ph_default_params.restype = None
    lib.chase_ph_create.argtypes = [C.POINTER(Params), vp, vp, i64, vp, C.POINTER(vp)]
    lib.chase_ph_destroy.argtypes = [vp]
    lib.chase_ph_last_error.argtypes = [vp]
    lib.chase_ph_last_error.restype = C.c_char_p
    lib.chase_ph_apply_h.argtypes = [vp, i32, vp, i64, vp, i64, i32]
    lib.chase_ph_filter.argtypes = [vp, i32, vp, i64, pi, dbl, dbl, dbl, i32]
    lib.chase_ph_filter_refined.argtypes = [vp, i32, vp, i64, vp, i64, pd, pi, dbl, dbl, dbl]
    lib.chase_ph_qr.argtypes = [vp, i32, vp, i64, vp, i64, pi]
    lib.chase_ph_oblique_rr.argtypes = [vp, i32, vp, i64, pd, vp, i64, vp, i64]
    lib.chase_ph_oblique_rr_backup.argtypes = [vp, i32, vp, i64, pd, vp, i64, vp, i64]
    lib.chase_ph_oblique_rr_general.argtypes = [vp, i32, vp, i64, pd, vp, i64, vp, i64]
    lib.chase_ph_residuals.argtypes = [vp, i32, i32, vp, i64, vp, i64, vp, i64, pd, vp, i64, pd]
    lib.chase_ph_solve.argtypes = [vp, vp, i64, vp, i64, pd, vp, i64, pd, C.POINTER(Info)]
    lib.chase_ph_eigval_backward.argtypes = [vp, i32, vp, i64, pd, vp, vp, i64]
    lib.chase_ph_eigval_backward_noalloc.argtypes = [i64, i32, vp, i64, pd, vp, vp, i64, vp]
    lib.chase_ph_last_timing.argtypes = [vp, pd, pi]
    lib.chase_ph_profile.argtypes = [vp, i32]
    lib.chase_ph_profile_read.argtypes = [vp, i32, pd, pd, pd, pi]
    lib.chase_ph_mfma_probe.argtypes = [i32, i32, pd]
    for name in EXPORTS:
        fn = getattr(lib, name)
        if name not in ("chase_ph_default_params", "chase_ph_last_error"):
            fn.restype = C.c_int
    return lib
