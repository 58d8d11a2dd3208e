"""ctypes binding of libdemag.so (the C ABI declared in include/demag.h).

Argument marshalling only: every step of a field evaluation runs in the HIP
kernels of the library.  If the library has not been built, loading fails
loudly -- there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DEMAG_LIBRARY", os.path.join(_PKG, "libdemag.so"))

DEMAG_F32, DEMAG_F64 = 0, 1
STATUS = {0: "DEMAG_OK", -1: "DEMAG_EINVAL", -2: "DEMAG_ENOMEM", -3: "DEMAG_EHIP",
          -4: "DEMAG_EUNSUPPORTED", -5: "DEMAG_ESTATE"}

# name -> (restype, argtypes); mirrors include/demag.h
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
SIGNATURES = {
    "demag_plan_create": (_I, [ctypes.POINTER(_P), _I, _I, _I, _D, _D, _D, _I, _P]),
    "demag_plan_set_option": (_I, [_P, ctypes.c_char_p, _D]),
    "demag_plan_destroy": (_I, [_P]),
    "demag_plan_info": (_I, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "demag_field": (_I, [_P, _P, _D, _P, _P]),
    "demag_field_adjoint": (_I, [_P, _P, _D, _P, _I, _P]),
    "demag_field_energy": (_I, [_P, _P, _D, _P, _P, _P]),
    "demag_energy": (_I, [_P, _P, _D, ctypes.POINTER(_D), _P]),
    "demag_energy_async": (_I, [_P, _P, _D, _P, _P]),
    "demag_energy_gradient": (_I, [_P, _P, _D, _P, _P, _I, _P]),
    "demag_plan_spectrum": (_I, [_P, _P]),
    "demag_plan_tensor": (_I, [_P, _P]),
    "demag_plan_describe": (_I, [_P, ctypes.c_char_p, _I]),
    "demag_plan_pass_times": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_int64)]),
    "demag_autotune": (_I, [_P, _P]),
    "demag_batch_create": (_I, [ctypes.POINTER(_P), ctypes.POINTER(_P), _I, ctypes.POINTER(_P),
                                ctypes.POINTER(_P), _D, _P]),
    "demag_sp_prepare": (_I, [_P, _P]),
    "demag_sp_field": (_I, [_P, _P, _D, _P, _P]),
    "demag_sp_field_energy": (_I, [_P, _P, _D, _P, _P, _P]),
    "demag_sp_kernel": (_I, [_P, _P]),
    "demag_llg_heun": (_I, [_P, _P, _D, _D, _D, _D, _D, _D, _D, _I, _P, _P]),
    "demag_llg_heun_static": (_I, [_P, _P, _D, _D, _D, _D, _D, _D, _D, _I, _P]),
    "demag_tg_prepare": (_I, [_P, _P]),
    "demag_tg_field": (_I, [_P, _P, _D, _P, _P]),
    "demag_tg_field_energy": (_I, [_P, _P, _D, _P, _P, _P]),
    "demag_tg_info": (_I, [_P, _P]),
    "demag_tg_path": (_I, [_P, _P]),
    "demag_tg_sinc_nodes": (_I, [_D, _D, _D, _P, _P, _I]),
    "demag_tg_lowrank_prepare": (_I, [_P, _P]),
    "demag_tg_lowrank_field": (_I, [_P, _I, _I, _P, _P, _D, _P, _P, _P, _P]),
    "demag_tg_lowrank_info": (_I, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "demag_lowrank_compress": (_I, [_P, _I, _I, _I, _P, _P, _P, ctypes.POINTER(_D), _P]),
    "demag_batch_autotune": (_I, [_P, _P]),
    "demag_batch_launch": (_I, [_P, _P]),
    "demag_batch_info": (_I, [_P, _P]),
    "demag_batch_destroy": (_I, [_P]),
    "demag_last_error": (ctypes.c_char_p, []),
}

_lib = None


class DemagError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} -> {STATUS.get(code, code)}: {msg}")
        self.code = code


def load(path: str | None = None):
    """Load libdemag.so and declare its signatures (cached)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build the HIP library first "
                          "(python -m paper_1204_4302_amd.build)")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def check(fn: str, code: int):
    if code != 0:
        msg = load().demag_last_error().decode(errors="replace")
        raise DemagError(fn, code, msg)


def call(fn: str, *args):
    check(fn, getattr(load(), fn)(*args))
