"""ctypes binding of libtoeplitz.so (the C ABI in include/toeplitz.h).

Argument marshalling only: every step of apply and solve runs in the library's
HIP kernels.  Loading fails loudly if the library has not been built; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# TOEPLITZ_LIBRARY may name another build of the same library (e.g. one
# compiled with different tuning flags); the default is the in-tree build.
LIB_PATH = os.environ.get("TOEPLITZ_LIBRARY") or os.path.join(_HERE, "libtoeplitz.so")

TP_OK, TP_E_INVAL, TP_E_NOMEM, TP_E_HIP, TP_E_NOCONV, TP_E_BREAKDOWN, TP_E_UNSUPPORTED = range(7)
TP_FP64, TP_FP32, TP_MIXED = 0, 1, 2
STATUS_NAMES = {0: "TP_OK", 1: "TP_E_INVAL", 2: "TP_E_NOMEM", 3: "TP_E_HIP", 4: "TP_E_NOCONV",
                5: "TP_E_BREAKDOWN", 6: "TP_E_UNSUPPORTED"}
PREC = {"fp64": TP_FP64, "fp32": TP_FP32, "mixed": TP_MIXED}

# every symbol the header declares
EXPORTS = ("toeplitz_plan_bytes", "toeplitz_plan_create", "toeplitz_plan_info", "toeplitz_matvec",
           "toeplitz_matvec_profile",
           "toeplitz_solve_opts_default", "toeplitz_solve", "toeplitz_plan_spectrum", "toeplitz_plan_destroy",
           "toeplitz_last_error", "toeplitz_batch_begin", "toeplitz_batch_admit", "toeplitz_batch_release",
           "toeplitz_batch_step", "toeplitz_batch_poll", "toeplitz_batch_end", "toeplitz_port_smatrix",
           "toeplitz_far_field", "toeplitz_precond_bytes", "toeplitz_precond_create", "toeplitz_precond_apply",
           "toeplitz_precond_bytes_for", "toeplitz_gen_symmetric", "toeplitz_schur_bytes", "toeplitz_schur_create", "toeplitz_schur_solve",
           "toeplitz_matvec_static", "toeplitz_static_scratch_bytes", "toeplitz_plan_bytes_placed",
           "toeplitz_plan_create_placed", "toeplitz_plan_set_option", "toeplitz_plan_get_option", "toeplitz_tune",
           "toeplitz_stage_time", "toeplitz_plan_path")
TP_SYM_RIM, TP_SYM_GEN = 1, 2
TP_OPT_SPECTRUM_PASS, TP_OPT_MFMA_COLS, TP_OPT_MFMA_MIN_R, TP_OPT_FFT2_LDS, TP_OPT_MULTI_FUSED = 1, 2, 3, 4, 5
TP_OPT_PROD_LDS, TP_OPT_RIM_OVERLAP, TP_OPT_DUAL_LAUNCH = 6, 7, 8
TP_PASS_AUTO, TP_PASS_FUSED, TP_PASS_PAIRS = 0, 1, 2
PATH_BITS = {"fused": 1, "pairs": 2, "mfma": 4, "dense_rim": 8, "rim_mfma": 16, "tiles2d": 32, "persistent": 64,
             "rim_overlap": 128, "joined": 256}


class PlanDesc(ctypes.Structure):
    _fields_ = [("Nx", ctypes.c_int), ("Ny", ctypes.c_int), ("b", ctypes.c_int), ("Nr", ctypes.c_int),
                ("Px", ctypes.c_int), ("Py", ctypes.c_int), ("N", ctypes.c_long), ("Nt", ctypes.c_long),
                ("max_rhs", ctypes.c_int), ("restart", ctypes.c_int), ("prec", ctypes.c_int),
                ("spectrum_bytes", ctypes.c_size_t), ("rim_bytes", ctypes.c_size_t),
                ("workspace_bytes", ctypes.c_size_t), ("total_bytes", ctypes.c_size_t),
                ("reciprocal", ctypes.c_int), ("half_spectrum", ctypes.c_int), ("nrc", ctypes.c_int),
                ("bc", ctypes.c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("mode", ctypes.c_int), ("x0_given", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("precond", ctypes.c_int)]


class TuneResult(ctypes.Structure):
    _fields_ = [("spectrum_pass", ctypes.c_int), ("mfma_cols", ctypes.c_int), ("fft2_lds", ctypes.c_int),
                ("multi_fused", ctypes.c_int), ("prod_lds", ctypes.c_int), ("rim_overlap", ctypes.c_int),
                ("candidates", ctypes.c_int), ("ms", ctypes.c_double),
                ("ms_default", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("status", ctypes.c_int),
                ("relres", ctypes.c_double)]


class ToeplitzError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded library; raises if libtoeplitz.so is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        # torch first: it loads the HIP runtime the library then shares (the
        # library loaded first would bring its own copy in ahead of torch's)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, ci, cl, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_size_t
        L.toeplitz_plan_bytes.argtypes = [ci, ci, ci, ci, ci, ci, ci, ci, ctypes.POINTER(sz)]
        L.toeplitz_gen_symmetric.argtypes = [ci, ci, ci, vp, ctypes.POINTER(ci)]
        L.toeplitz_schur_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        L.toeplitz_schur_create.argtypes = [vp, vp, vp, sz, ctypes.POINTER(SolveOpts), vp]
        L.toeplitz_schur_solve.argtypes = [vp, vp, vp, cl, vp, cl, ci, ctypes.POINTER(SolveOpts),
                                           ctypes.POINTER(SolveInfo), vp]
        L.toeplitz_plan_create.argtypes = [ci, ci, ci, ci, vp, vp, vp, vp, ci, ci, ci, vp, sz, vp,
                                           ctypes.POINTER(vp)]
        L.toeplitz_plan_bytes_placed.argtypes = [ci, ci, ci, ci, ci, ci, ci, ci, ci, ctypes.POINTER(sz)]
        L.toeplitz_plan_create_placed.argtypes = [ci, ci, ci, ci, vp, vp, vp, vp, vp, ci, ci, ci, ci, vp, sz, vp,
                                                  ctypes.POINTER(vp)]
        L.toeplitz_plan_set_option.argtypes = [vp, ci, ci]
        L.toeplitz_stage_time.argtypes = [vp, ci, vp, cl, vp, cl, ci, ci, ci, vp, ctypes.POINTER(ctypes.c_double)]
        L.toeplitz_plan_path.argtypes = [vp, ci, ci, ci, ctypes.POINTER(ci)]
        L.toeplitz_tune.argtypes = [vp, ci, vp, cl, vp, cl, ci, ci, vp, ctypes.POINTER(TuneResult)]
        L.toeplitz_plan_get_option.argtypes = [vp, ci, ctypes.POINTER(ci)]
        L.toeplitz_plan_info.argtypes = [vp, ctypes.POINTER(PlanDesc)]
        L.toeplitz_matvec.argtypes = [vp, ci, vp, cl, vp, cl, ci, vp]
        L.toeplitz_matvec_static.argtypes = [vp, ci, vp, cl, vp, cl, ci, vp]
        L.toeplitz_static_scratch_bytes.argtypes = []
        L.toeplitz_static_scratch_bytes.restype = sz
        L.toeplitz_matvec_profile.argtypes = [vp, ci, vp, cl, vp, cl, ci, ci, vp, ctypes.POINTER(ctypes.c_double)]
        L.toeplitz_solve_opts_default.argtypes = [ctypes.POINTER(SolveOpts)]
        L.toeplitz_solve_opts_default.restype = None
        L.toeplitz_solve.argtypes = [vp, vp, cl, vp, cl, ci, ctypes.POINTER(SolveOpts),
                                     ctypes.POINTER(SolveInfo), vp]
        L.toeplitz_plan_spectrum.argtypes = [vp, ci, ci, ci, vp]
        L.toeplitz_batch_begin.argtypes = [vp, ctypes.POINTER(SolveOpts)]
        L.toeplitz_batch_admit.argtypes = [vp, ci, vp, vp, ctypes.c_double, ci, vp]
        L.toeplitz_batch_release.argtypes = [vp, ci]
        L.toeplitz_batch_step.argtypes = [vp, ci]
        L.toeplitz_batch_poll.argtypes = [vp, ci, ci, ctypes.POINTER(ci), ctypes.POINTER(SolveInfo)]
        L.toeplitz_batch_end.argtypes = [vp]
        cd = ctypes.c_double
        L.toeplitz_port_smatrix.argtypes = [ci, cl, vp, cl, vp, vp, cd, vp, cl, vp, sz, vp]
        L.toeplitz_far_field.argtypes = [ci, ci, ci, ci, cd, cd, vp, vp, vp, vp, vp, cl, ci, vp, ci, cd, cd, vp, vp]
        L.toeplitz_precond_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        L.toeplitz_precond_bytes_for.argtypes = [ci, ci, ci, ci, ci, ci, ctypes.POINTER(sz)]
        L.toeplitz_precond_create.argtypes = [vp, vp, sz, vp]
        L.toeplitz_precond_apply.argtypes = [vp, ci, vp, cl, vp, cl, ci, vp]
        L.toeplitz_plan_destroy.argtypes = [vp]
        L.toeplitz_plan_destroy.restype = None
        L.toeplitz_last_error.restype = ctypes.c_char_p
        for name in ("toeplitz_plan_bytes", "toeplitz_plan_create", "toeplitz_plan_info", "toeplitz_matvec",
                     "toeplitz_matvec_profile",
                     "toeplitz_solve", "toeplitz_plan_spectrum", "toeplitz_batch_begin", "toeplitz_batch_admit",
                     "toeplitz_batch_release", "toeplitz_batch_step", "toeplitz_batch_poll", "toeplitz_batch_end",
                     "toeplitz_port_smatrix", "toeplitz_far_field", "toeplitz_precond_bytes",
                     "toeplitz_precond_bytes_for", "toeplitz_precond_create", "toeplitz_precond_apply", "toeplitz_gen_symmetric",
                     "toeplitz_schur_bytes", "toeplitz_schur_create", "toeplitz_schur_solve",
           "toeplitz_matvec_static", "toeplitz_static_scratch_bytes"):
            getattr(L, name).restype = ci
        _lib = L
    return _lib


def check(status):
    if status != TP_OK:
        raise ToeplitzError(status, lib().toeplitz_last_error().decode())
    return status
