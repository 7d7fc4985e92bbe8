"""ctypes mirror of include/dda.h.  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdda.so")

DDA_OK = 0
DDA_E_INVALID = 1
DDA_E_NOMEM = 2
DDA_E_DEVICE = 3
DDA_E_NOT_CONVERGED = 4
DDA_E_BREAKDOWN = 5
DDA_E_NONFINITE = 6

STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_NOT_CONVERGED",
                5: "E_BREAKDOWN", 6: "E_NONFINITE"}

DDA_LATTDR = 0
DDA_GKDLDR = 1
DDA_BICGSTAB = 0
DDA_QMR_SYM = 1
DDA_BICGSTAB2 = 2
DDA_FP64 = 0
DDA_FP32_MATVEC = 1
DDA_FLAG_RECOMPUTE_GREEN = 1
DDA_FLAG_NO_FINAL_CHECKS = 2
DDA_FLAG_NO_AUTOTUNE = 4
DDA_FLAG_NO_GRAPH = 8
DDA_FLAG_SEPARATE_TARGETS = 16


class C64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Incidence(ctypes.Structure):
    _fields_ = [("khat", ctypes.c_double * 3), ("e0", C64 * 3)]


class Opts(ctypes.Structure):
    _fields_ = [
        ("wavelength", ctypes.c_double),
        ("aeff", ctypes.c_double),
        ("m_medium", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("polarizability", ctypes.c_int32),
        ("solver", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("kernel_variant", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("qext", ctypes.c_double),
        ("qabs", ctypes.c_double),
        ("qsca", ctypes.c_double),
        ("qpha", ctypes.c_double),
        ("rel_residual", ctypes.c_double),
        ("normal_eq_residual", ctypes.c_double),
        ("kd", ctypes.c_double),
        ("aeff_d", ctypes.c_double),
        ("iters", ctypes.c_int32),
        ("matvecs", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("refinements", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


# name -> (restype, argtypes): every symbol include/dda.h declares
VP = ctypes.c_void_p
SIGNATURES = {
    "dda_ctx_create": (ctypes.c_int, [ctypes.c_int, VP, ctypes.POINTER(VP)]),
    "dda_ctx_destroy": (ctypes.c_int, [VP]),
    "dda_target_create": (ctypes.c_int, [VP, ctypes.c_int64, VP, VP, ctypes.POINTER(VP)]),
    "dda_target_destroy": (ctypes.c_int, [VP]),
    "dda_target_geometry": (ctypes.c_int, [VP, VP, VP]),
    "dda_apply": (ctypes.c_int, [VP, VP, ctypes.POINTER(Opts), ctypes.c_int32, ctypes.POINTER(Incidence), VP, VP]),
    "dda_apply_noalloc": (ctypes.c_int, [VP, VP, ctypes.POINTER(Opts), ctypes.c_int32, ctypes.POINTER(Incidence), VP,
                                         VP]),
    "dda_solve": (ctypes.c_int, [VP, VP, ctypes.POINTER(Opts), ctypes.c_int32, ctypes.POINTER(Incidence), VP, VP,
                                 ctypes.POINTER(Result)]),
    "dda_solve_rhs": (ctypes.c_int, [VP, VP, ctypes.POINTER(Opts), ctypes.c_int32, ctypes.POINTER(Incidence), VP, VP,
                                     VP, ctypes.POINTER(Result)]),
    "dda_solve_batched": (ctypes.c_int, [VP, ctypes.c_int32, VP, ctypes.POINTER(Opts), ctypes.c_int32, VP,
                                         ctypes.POINTER(Incidence), VP, ctypes.POINTER(Result)]),
    "dda_grad_eps": (ctypes.c_int, [VP, VP, ctypes.POINTER(Opts), ctypes.POINTER(Incidence), VP, ctypes.c_double,
                                    ctypes.c_double, VP, ctypes.POINTER(Result)]),
    "dda_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdda.so (built in-tree by ``paper_1202_3424_amd.build``).  Raises
    if it is missing: there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1202_3424_amd.build.build() "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


DDA_TIMING_CATEGORIES = 8
TIMING_NAMES = ["scatter_fft_x", "fft_y_fwd", "fft_z_green", "fft_y_inv", "fft_x_gather", "krylov", "green_setup",
                "setup"]


class Timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * DDA_TIMING_CATEGORIES), ("launches", ctypes.c_int64 * DDA_TIMING_CATEGORIES),
                ("all_launches", ctypes.c_int64 * DDA_TIMING_CATEGORIES)]


SIGNATURES["dda_ctx_set_timing"] = (ctypes.c_int, [VP, ctypes.c_int])
SIGNATURES["dda_ctx_get_timing"] = (ctypes.c_int, [VP, ctypes.POINTER(Timing)])
SIGNATURES["dda_ctx_set_timing_sample"] = (ctypes.c_int, [VP, ctypes.c_int])
SIGNATURES["dda_far_field"] = (ctypes.c_int, [VP, VP, ctypes.POINTER(Opts), ctypes.c_int32, VP, ctypes.c_int32, VP,
                                              VP, VP, VP, VP])
SIGNATURES["dda_scattering_averages"] = (ctypes.c_int, [VP, VP, ctypes.POINTER(Opts), ctypes.c_int32,
                                                        ctypes.POINTER(Incidence), VP, ctypes.c_int32,
                                                        ctypes.c_int32, VP])
SIGNATURES["dda_mueller"] = (ctypes.c_int, [ctypes.c_int32, VP, VP, VP, VP, VP, VP])
SIGNATURES["dda_nearfield_volume"] = (ctypes.c_int, [VP, VP, VP, VP])
SIGNATURES["dda_nearfield"] = (ctypes.c_int, [VP, VP, ctypes.POINTER(Opts), VP, ctypes.c_int32,
                                              ctypes.POINTER(Incidence), VP, VP, VP])
SIGNATURES["dda_field_line"] = (ctypes.c_int, [VP, ctypes.c_int32, VP, VP, VP, VP, VP, ctypes.c_int32, VP])
SIGNATURES["dda_ctx_tuned_variants"] = (ctypes.c_int, [VP, VP, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(ctypes.c_int32)])
