"""ctypes loader for libvp.so (the HIP C ABI declared in include/vp.h).

Loading fails loudly: there is no CPU fallback for any entry point."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvp.so")

VP_OK = 0
VP_EINVAL = -1
VP_EUNSUPPORTED = -2
VP_ELAUNCH = -3
VP_INCLUDE_ZERO = 1
VP_PATHS_PER_VECTOR = 2
VP_DEMAP_REGION = 4
VP_SE_EXACT = 0
VP_SE_EXHAUSTED = 1
VP_SE_NONE = 2
VP_NOALLOC_MAX_VECTORS = 65536

_lib = None


class VPError(RuntimeError):
    def __init__(self, code: int, fn: str):
        msg = _lib.vp_strerror(code).decode() if _lib is not None else str(code)
        extra = ""
        if code == VP_ELAUNCH and _lib is not None:
            extra = f" (hipError {_lib.vp_last_hip_error()})"
        super().__init__(f"{fn}: {msg}{extra}")
        self.code = code


_P = ctypes.c_void_p
_I = ctypes.c_int
_F = ctypes.c_float

SIGNATURES = {
    "vp_preprocess": [_P, _I, _I, _I, _F, _P, _P, _P, _P, _P, _P],
    "vp_preprocess_unsorted": [_P, _I, _I, _I, _F, _P, _P, _P, _P, _P, _P],
    "vp_paths_mop": [_P, _I, _I, _I, _P, _P, _P],
    "vp_search": [_P, _P, _P, _P, _P, _P, _I, ctypes.c_int64, _I, _I, _I, ctypes.c_uint32, _P, _P, _P, _P],
    "vp_search_fallback": [_P, _P, _P, _P, _P, _P, _I, ctypes.c_int64, _I, _I, _I, ctypes.c_uint32, _P, _F,
                           ctypes.c_int32, _P, _P, _P, _P, _P],
    "vp_search_fallback_noalloc": [_P, _P, _P, _P, _P, _P, _I, ctypes.c_int64, _I, _I, _I, ctypes.c_uint32, _P,
                                   _F, ctypes.c_int32, _P, _P, _P, _P],
    "vp_precode": [_P, _P, _P, _P, _P, _I, _I, _I, _I, _F, _P, _P],
    "vp_apply_user_tau": [_P, _P, _I, _I, _I, _I, _P, _P, _P, _P, _P, _P],
    "vp_sphere_encode": [_P, _P, _P, _F, _I, _I, _I, _P, ctypes.c_int64, _P, _P, _P, _P, _P],
    "vp_fx_quantize": [_P, _P, _P, _P, _I, _I, _I, _I, _P, _P, _P, _P],
    "vp_fx_search": [_P, _P, _P, _P, _P, _I, ctypes.c_int64, _I, _I, _I, _I, ctypes.c_uint32, _P, _P, _P, _P],
    "vp_strerror": [_I],
    "vp_last_hip_error": [],
    "vp_version": [],
}


def load(path: str = LIB_PATH):
    """Load libvp.so and bind every exported entry point's signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2602_12098_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, argtypes in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = _I
    lib.vp_strerror.restype = ctypes.c_char_p
    lib.vp_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(code: int, fn: str) -> None:
    if code != VP_OK:
        raise VPError(code, fn)
