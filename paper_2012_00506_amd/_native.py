"""ctypes declarations of the C ABI in include/feastband.h."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# FEASTBAND_LIB names another build of the same library (the host-sanitizer
# build of the C ABI checks); it is never a substitute for the GPU code
LIB_PATH = os.environ.get("FEASTBAND_LIB") or os.path.join(_HERE, "libfeastband.so")

FB_REAL64 = 1
FB_COMPLEX128 = 2
FB_PLAN_EQUAL_WIDTH = 0
FB_PLAN_EQUAL_COUNT = 1
FB_PLAN_LEARNED = 2
PROF_CLASSES = ["lu", "invert", "solve", "resid", "inertia", "jacobi", "gemm", "bandmm"]


PI32 = C.POINTER(C.c_int32)


class fb_band(C.Structure):
    _fields_ = [("n", C.c_int64), ("b", C.c_int32), ("dtype", C.c_int32),
                ("ldab", C.c_int64), ("ab", C.c_void_p)]


class fb_solve_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("ir_tol", C.c_double), ("ir_max", C.c_int32),
                ("tile", C.c_int32)]


class fb_feast_opts(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("ir_tol", C.c_double), ("ir_max", C.c_int32),
                ("batched", C.c_int32), ("hbm_budget", C.c_double), ("pairs", C.c_int32),
                ("rule", C.c_int32), ("ratio", C.c_double), ("tune_cache", C.c_char_p),
                ("graph", C.c_int32), ("ir_from", C.c_double)]


class fb_plan_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("K", C.c_int32), ("lo", C.c_double), ("hi", C.c_double),
                ("count_tol", C.c_double), ("cert_delta", C.c_double),
                ("max_rounds", C.c_int32), ("planner", C.c_void_p), ("seed", C.c_uint64),
                ("nev", C.c_int64), ("targets", PI32)]


class fb_prev_opts(C.Structure):
    _fields_ = [("K", C.c_int32), ("nev", C.c_int64), ("alpha", C.c_double), ("m1", C.c_int32),
                ("cert_delta", C.c_double), ("max_sweeps", C.c_int32), ("max_steps", C.c_int32)]


P = C.c_void_p
PI64 = C.POINTER(C.c_int64)
PD = C.POINTER(C.c_double)
PSZ = C.POINTER(C.c_size_t)

# name -> (restype, argtypes); every symbol declared in include/feastband.h
SIGNATURES = {
    "band_inertia": (C.c_int, [C.POINTER(fb_band), C.c_int32, PD, PI32, PI32, PI32, P, PSZ, P]),
    "band_inertia_noalloc": (C.c_int, [C.POINTER(fb_band), C.c_int32, PD, PI32, PI32, PI32, P]),
    "band_shifted_solve": (C.c_int, [C.POINTER(fb_band), C.c_int32, PD, PI32, C.POINTER(P), PI64,
                                     C.POINTER(P), C.POINTER(P), PI64, PD, PI32,
                                     C.POINTER(fb_solve_opts), P, PSZ, P]),
    "feast_band_slice": (C.c_int, [C.POINTER(fb_band), C.c_int32, PD, PD, PI32, PI32,
                                   C.POINTER(P), PI64, C.POINTER(P), C.POINTER(P), PI32, PI32,
                                   PI32, C.POINTER(fb_feast_opts), P, PSZ, P]),
    "slice_plan": (C.c_int, [C.POINTER(fb_band), C.POINTER(fb_plan_opts), PD, PI32, PI32, P,
                             PSZ, P]),
    "slice_plan_prev": (C.c_int, [C.POINTER(fb_band), PD, C.c_int64, C.POINTER(fb_prev_opts), PD,
                                  PI32, PI32, PI32, P, PSZ, P]),
    "slice_certify": (C.c_int, [C.POINTER(fb_band), C.c_int32, PD, C.c_double, PI32, PI32, PI32,
                                PI32, P, PSZ, P]),
    "fb_m0_rule": (C.c_int32, [C.c_int32]),
    "feast_filter": (C.c_int, [C.POINTER(fb_band), C.c_int32, PD, PD, PI32, C.POINTER(P), PI64,
                               C.POINTER(P), PI64, PD, PI32, C.POINTER(fb_feast_opts), P, PSZ, P]),
    "band_rayleigh_ritz": (C.c_int, [C.POINTER(fb_band), C.c_int32, PI32, C.POINTER(P), PI64,
                                     C.POINTER(P), PI64, C.POINTER(P), C.POINTER(P), PI32, PI32, P,
                                     PSZ, P]),
    "fb_profile_enable": (C.c_int, [C.c_int32]),
    "fb_profile_read": (C.c_int, [C.c_int32, PI64, PD, PD]),
    "fb_autotune": (C.c_int, [C.POINTER(fb_band), C.c_int32, C.c_int32, C.c_int32, C.c_char_p,
                              PI32, PD, P, PSZ, P]),
    "fb_tune_load": (C.c_int, [C.c_char_p]),
    "band_cheb_moments": (C.c_int, [C.POINTER(fb_band), C.c_int32, C.c_int32, C.c_uint64, PD, PD,
                                    P, PSZ, P]),
    "band_features": (C.c_int, [C.POINTER(fb_band), C.c_uint64, PD, P, PSZ, P]),
    "fb_planner_bytes": (C.c_size_t, []),
    "planner_forward": (C.c_int, [P, C.c_int32, P, P, P, PSZ, P]),
    "planner_train_step": (C.c_int, [P, P, C.c_int32, P, P, C.c_float, C.c_int32,
                                     C.POINTER(C.c_float), P, P, PSZ, P]),
    "fb_strerror": (C.c_char_p, [C.c_int]),
    "fb_contour": (C.c_int, [C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_double, PD, PD]),
    "fb_device_info": (C.c_int, [PI32, C.c_char_p, C.c_int32]),
}

_lib = None


class FeastBandError(RuntimeError):
    def __init__(self, func: str, code: int, msg: str):
        super().__init__(f"{func} failed with code {code}: {msg}")
        self.code = code


def lib():
    """Load libfeastband.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with paper_2012_00506_amd.build.build() "
                "(the GPU path has no fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(func: str, code: int, allow_positive: bool = False) -> int:
    if code == 0 or (allow_positive and code > 0):
        return code
    msg = lib().fb_strerror(code).decode()
    raise FeastBandError(func, code, msg)
