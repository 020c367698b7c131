"""ctypes binding of libdsnlm.so (argument marshalling only).

The library is loaded from this package directory.  There is no fallback:
if the HIP library has not been built, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsnlm.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {
    0: "DSNLM_OK", -1: "DSNLM_EINVAL", -2: "DSNLM_ENOMEM", -3: "DSNLM_EDEVICE",
    -4: "DSNLM_ENONFINITE", -5: "DSNLM_EUNSUPPORTED",
}

LADMM_OP_SR = 1
LADMM_OP_SPI = 2


class DsnlmImage(C.Structure):
    _fields_ = [
        ("guide", C.c_void_p),
        ("x", C.c_void_p),
        ("y", C.c_void_p),
        ("n1", C.c_int),
        ("n2", C.c_int),
        ("h", C.c_float),
    ]


class DsnlmImageGrad(C.Structure):
    _fields_ = [
        ("dy", C.c_void_p),
        ("dx", C.c_void_p),
        ("dguide", C.c_void_p),
        ("dh", C.c_void_p),
    ]


class LadmmOperator(C.Structure):
    _fields_ = [
        ("kind", C.c_int),
        ("n1", C.c_int),
        ("n2", C.c_int),
        ("taps", C.POINTER(C.c_float)),
        ("blur_size", C.c_int),
        ("factor", C.c_int),
        ("boundary", C.c_int),
        ("y", C.c_void_p),
        ("ones", C.c_void_p),
        ("K", C.c_int),
        ("eta", C.c_float),
        ("t_min", C.c_float),
    ]


class LadmmParams(C.Structure):
    _fields_ = [
        ("lam", C.c_float),
        ("rho", C.c_float),
        ("gamma", C.c_float),
        ("S", C.c_int),
        ("P", C.c_int),
        ("h", C.c_float),
        ("iters", C.c_int),
        ("freeze_after", C.c_int),
        ("lo", C.c_float),
        ("hi", C.c_float),
        ("denoiser", C.c_int),
    ]


class DsnlmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"HIP library {LIB_PATH} is missing; build it with "
            "`python -m paper_1901_06110_amd.build` (there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    vp, i, f = C.c_void_p, C.c_int, C.c_float
    pp = C.POINTER(C.c_void_p)
    sig = {
        "dsnlm_build_weights": (i, [vp, i, i, i, i, f, vp, pp]),
        "dsnlm_apply": (i, [vp, vp, vp, vp]),
        "dsnlm_forward": (i, [vp, vp, vp, i, i, i, i, f, vp, pp]),
        "dsnlm_forward_noalloc": (i, [vp, vp, vp, i, i, i, i, f, vp]),
        "dsnlm_forward_noalloc_limit": (C.c_size_t, []),
        "dsnlm_forward_noalloc_bytes": (C.c_size_t, [i, i, i, i]),
        "dsnlm_nlm": (i, [vp, vp, vp, i, i, i, i, f, vp, pp]),
        "dsnlm_forward_brute": (i, [vp, vp, vp, i, i, i, i, f, vp, pp]),
        "dsnlm_apply_backward": (i, [vp, vp, vp, vp, vp, vp, vp]),
        "dsnlm_weights_destroy": (None, [vp]),
        "dsnlm_weights_scalars": (i, [vp, C.POINTER(f), C.POINTER(i), vp]),
        "dsnlm_weights_array": (vp, [vp, i]),
        "dsnlm_forward_batched": (i, [C.POINTER(DsnlmImage), i, i, i, vp]),
        "dsnlm_backward_batched": (i, [C.POINTER(DsnlmImageGrad), i, vp]),
        "dsnlm_batched_state": (i, [i, C.POINTER(f), C.POINTER(i), pp, pp, vp]),
        "ladmm_step": (i, [C.POINTER(LadmmOperator), C.POINTER(LadmmParams), i, pp, vp, vp, vp, vp]),
        "ladmm_solve": (i, [C.POINTER(LadmmOperator), C.POINTER(LadmmParams), vp, vp, vp, vp, vp, vp]),
        "ladmm_apply_forward": (i, [C.POINTER(LadmmOperator), vp, vp, vp]),
        "admm_cg_solve": (i, [C.POINTER(LadmmOperator), C.POINTER(LadmmParams), i, vp, vp, vp, vp, vp]),
        "ladmm_step_backward": (i, [C.POINTER(LadmmOperator), C.POINTER(LadmmParams), i, vp, vp, vp, vp, vp,
                                    vp, vp, vp, vp, vp, vp, vp]),
        "ladmm_solve_backward": (i, [C.POINTER(LadmmOperator), C.POINTER(LadmmParams), vp, vp, vp, vp, vp,
                                     vp, vp, vp, vp, vp]),
        "ladmm_gradient": (i, [C.POINTER(LadmmOperator), vp, vp, vp]),
        "ladmm_operator_norm2": (i, [C.POINTER(LadmmOperator), i, C.POINTER(f), vp]),
        "dsnlm_tune_set": (i, [i, i, i, i]),
        "dsnlm_tune_get": (i, [i, i, i, C.POINTER(i)]),
        "dsnlm_tune": (i, [vp, i, i, i, i, f, i, vp]),
        "dsnlm_tune_set_groups": (i, [i, i, i, i, i]),
        "dsnlm_tune_get_groups": (i, [i, i, i, i, C.POINTER(i)]),
        "dsnlm_peak_probe": (i, [i, C.POINTER(C.c_double), vp]),
        "dsnlm_profile_enable": (i, [i]),
        "dsnlm_profile_query": (i, [i, C.POINTER(C.c_double), C.POINTER(i)]),
        "dsnlm_profile_reset": (i, []),
        "dsnlm_last_error": (C.c_char_p, []),
        "dsnlm_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def get():
    """The loaded library (loaded on first use; raises if it was not built)."""
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB

EXPORTED = [
    "dsnlm_build_weights", "dsnlm_apply", "dsnlm_forward", "dsnlm_apply_backward",
    "dsnlm_weights_destroy", "dsnlm_weights_scalars", "dsnlm_weights_array",
    "dsnlm_forward_batched", "ladmm_step", "ladmm_solve", "ladmm_apply_forward",
    "ladmm_gradient", "ladmm_operator_norm2", "dsnlm_last_error", "dsnlm_version",
    "dsnlm_profile_enable", "dsnlm_profile_query", "dsnlm_profile_reset",
    "dsnlm_tune_set", "dsnlm_tune_get", "dsnlm_tune", "dsnlm_peak_probe",
    "ladmm_step_backward", "ladmm_solve_backward", "dsnlm_backward_batched", "dsnlm_nlm",
    "dsnlm_forward_brute", "admm_cg_solve", "dsnlm_batched_state",
    "dsnlm_forward_noalloc", "dsnlm_forward_noalloc_limit", "dsnlm_forward_noalloc_bytes",
    "dsnlm_tune_set_groups", "dsnlm_tune_get_groups",
]

K_PASS_A, K_PASS_B, K_APPLY, K_EPILOGUE, K_BWD_PREP, K_PASS_C, K_PASS_D, K_BWD_TAIL, K_LADMM, K_HALF_AUX = range(10)


def check(code: int) -> None:
    if code != OK:
        raise DsnlmError(code, get().dsnlm_last_error().decode())
