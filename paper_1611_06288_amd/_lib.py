"""ctypes declarations of the C ABI in ``include/pfc.h`` (argument marshalling only).

The HIP library is loaded from the package folder; there is no fallback:
if ``libpfc_hip.so`` is missing every call raises ``HipLibraryMissing``.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpfc_hip.so")

PFC_OK = 0
PFC_ERR_INVALID_ARG = 1
PFC_ERR_NOT_CONVERGED = 2
PFC_ERR_NONFINITE = 3
PFC_ERR_HIP = 4
PFC_ERR_OOM = 5

PFC_FP64, PFC_MIXED = 0, 1
PFC_CYCLE_V, PFC_CYCLE_F = 0, 1
PFC_LIN_NEWTON, PFC_LIN_PICARD = 0, 1
PFC_SWEEP_FULL = 2
PFC_MOBILITY_ONE, PFC_MOBILITY_QUADRATIC = 0, 1
PFC_SCHEME_CS2, PFC_SCHEME_CS1 = 0, 1
PFC_ENERGY_STATIC_MAX_N = 1024

PFC_KERNEL_SMOOTH0 = 0
PFC_KERNEL_RESIDUAL0 = 1
PFC_KERNEL_PROLONG0 = 2
PFC_KERNEL_NORM0 = 3
PFC_KERNEL_COARSE = 4
PFC_KERNEL_SWEEP_NORM0 = 5
PFC_KERNEL_COUNT = 6
KERNEL_NAMES = ["smooth0", "residual0", "prolong0", "norm0", "coarse", "sweep_norm0"]


class HipLibraryMissing(RuntimeError):
    pass


class PfcConfig(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32), ("max_cycles", C.c_int32),
        ("cycle", C.c_int32), ("lin", C.c_int32), ("precision", C.c_int32), ("mobility", C.c_int32),
        ("L", C.c_double), ("eps", C.c_double), ("dt", C.c_double), ("tol", C.c_double),
        ("mob_m0", C.c_double), ("mob_m1", C.c_double), ("mob_m2", C.c_double),
        ("mob_min", C.c_double), ("scheme", C.c_int32),
    ]


class PfcStepInfo(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("status", C.c_int32),
                ("res0", C.c_double), ("res_final", C.c_double)]


_lib = None

# name -> (restype, argtypes)
_vp, _dp, _i32, _d = C.c_void_p, C.c_void_p, C.c_int32, C.c_double
SIGNATURES = {
    "pfc_create": (_i32, [C.POINTER(PfcConfig), _vp, C.POINTER(_vp)]),
    "pfc_destroy": (_i32, [_vp]),
    "pfc_set_stream": (_i32, [_vp, _vp]),
    "pfc_num_levels": (_i32, [_vp]),
    "pfc_level_size": (_i32, [_vp, _i32]),
    "pfc_init_guess": (_i32, [_vp, _dp, _dp, _dp]),
    "pfc_step": (_i32, [_vp, _dp, _dp, _dp, _dp, _dp, C.POINTER(PfcStepInfo)]),
    "pfc_run": (_i32, [_vp, _dp, _dp, _dp, _dp, _i32, C.POINTER(PfcStepInfo)]),
    "pfc_fas_vcycle": (_i32, [_vp, _dp, _dp, _dp, C.POINTER(C.c_double)]),
    "pfc_energy": (_i32, [_vp, _dp, _dp, C.POINTER(C.c_double)]),
    "pfc_energy_static": (_i32, [_i32, _d, _d, _dp, _dp, _dp, _vp]),
    "pfc_adjoint_step": (_i32, [_vp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _d, C.POINTER(_i32)]),
    "pfc_source": (_i32, [_vp, _dp, _dp, _dp]),
    "pfc_residual": (_i32, [_vp, _i32, _dp, _dp, _dp, _dp, C.POINTER(C.c_double)]),
    "pfc_smooth": (_i32, [_vp, _i32, _i32, _dp, _dp, _dp]),
    "pfc_restrict": (_i32, [_vp, _i32, _dp, _dp, _i32]),
    "pfc_prolong_add": (_i32, [_vp, _i32, _dp, _dp, _dp, _i32]),
    "pfc_coarse_solve": (_i32, [_vp, _dp, _dp, _dp, C.POINTER(_i32)]),
    "pfc_set_phistar": (_i32, [_vp, _i32, _dp]),
    "pfc_reset_coarse_cache": (_i32, [_vp]),
    "pfc_batch_create": (_i32, [_i32, C.POINTER(PfcConfig), _vp, C.POINTER(_vp)]),
    "pfc_batch_destroy": (_i32, [_vp]),
    "pfc_batch_set_state": (_i32, [_vp, _i32, _dp, _dp, _dp, _dp]),
    "pfc_batch_get_state": (_i32, [_vp, _i32, _dp, _dp, _dp, _dp]),
    "pfc_batch_run": (_i32, [_vp, _i32, C.POINTER(PfcStepInfo)]),
    "pfc_batch_init_state": (_i32, [_vp, _i32, _dp]),
    "pfc_batch_autotune": (_i32, [_vp, C.c_char_p, C.POINTER(_i32)]),
    "pfc_batch_last_error": (C.c_char_p, [_vp]),
    "pfc_timing_enable": (_i32, [_vp, _i32]),
    "pfc_timing_get": (_i32, [_vp, _i32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                              C.POINTER(C.c_double)]),
    "pfc_timing_reset": (_i32, [_vp]),
    "pfc_status_string": (C.c_char_p, [_i32]),
    "pfc_last_error": (C.c_char_p, [_vp]),
}


def lib():
    """Loads the HIP library (once).  Raises HipLibraryMissing if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HipLibraryMissing(
                f"{LIB_PATH} not found: build it with `python -m paper_1611_06288_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
