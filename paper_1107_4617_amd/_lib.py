"""ctypes binding of libbsk.so: argument marshalling only.

Every step of the filter runs in the HIP kernels of libbsk.so; this module
declares the C signatures of include/bsk.h and loads the in-tree library.  It
raises if the library is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsk.so")

BSK_OK = 0
BSK_EINVAL = -1
BSK_ERANGE = -2
BSK_ENOMEM = -3
BSK_EHIP = -4
BSK_EUNSUPPORTED = -5

BSK_FP32, BSK_BF16, BSK_FP16, BSK_FP64, BSK_I16 = 0, 1, 2, 3, 4
BSK_RANGE_COS, BSK_RANGE_POLY = 0, 1
RANGE_KERNELS = {"cos": BSK_RANGE_COS, "poly": BSK_RANGE_POLY}
PRECISIONS = {"fp32": BSK_FP32, "bf16": BSK_BF16, "fp16": BSK_FP16, "fp64": BSK_FP64, "i16": BSK_I16}

STATUS_NAMES = {0: "BSK_OK", -1: "BSK_EINVAL", -2: "BSK_ERANGE", -3: "BSK_ENOMEM", -4: "BSK_EHIP",
                -5: "BSK_EUNSUPPORTED"}

# Every symbol include/bsk.h declares.
EXPORTS = [
    "bilateral_shiftable", "bilateral_shiftable_ex", "bilateral_shiftable_noalloc", "bilateral_shiftable_nlm2", "bilateral_shiftable_train",
    "bilateral_shiftable_backward", "bilateral_shiftable_train_stack", "bilateral_shiftable_backward_stack",
    "bilateral_shiftable_batched", "bilateral_shiftable_batched_graph",
    "bsk_order_for", "bsk_plan_info", "bsk_truncation_error", "bsk_poly_order_for", "bsk_poly_plan_info",
    "bsk_autotune", "bsk_batched_shape", "bsk_autotune_batched", "bsk_tune_cache_load", "bsk_tune_cache_save",
    "bsk_tune_cache_clear", "bsk_set_workspace_limit", "bsk_last_error", "bsk_release", "bsk_version",
]


class Options(ctypes.Structure):
    _fields_ = [("order_mode", ctypes.c_int), ("N", ctypes.c_int), ("precision", ctypes.c_int),
                ("weight_eps", ctypes.c_double), ("kahan", ctypes.c_int), ("pitch_in", ctypes.c_int),
                ("pitch_out", ctypes.c_int), ("block", ctypes.c_int), ("strip_h", ctypes.c_int),
                ("order_chunk", ctypes.c_int), ("spatial_N", ctypes.c_int), ("spatial_sigma", ctypes.c_double),
                ("range_kernel", ctypes.c_int)]


class ImageDesc(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("out", ctypes.c_void_p), ("H", ctypes.c_int), ("W", ctypes.c_int),
                ("radius", ctypes.c_int), ("sigma_r", ctypes.c_float), ("N", ctypes.c_int)]


class BskError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

_vp = ctypes.c_void_p
_i = ctypes.c_int
_f = ctypes.c_float
_d = ctypes.c_double


def load():
    """Load the in-tree libbsk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "bilateral_shiftable": (_i, [_vp, _i, _i, _i, _f, _f, _vp]),
        "bilateral_shiftable_ex": (_i, [_vp, _i, _i, _i, _f, _f, _vp, ctypes.POINTER(Options), _vp]),
        "bilateral_shiftable_noalloc": (_i, [_vp, _i, _i, _i, _f, _f, _vp, ctypes.POINTER(Options), _vp]),
        "bilateral_shiftable_nlm2": (_i, [_vp, _i, _i, _i, _f, _f, _i, _i, _i, _i, _f, _vp, ctypes.POINTER(Options),
                                          _vp]),
        "bilateral_shiftable_train": (_i, [_vp, _i, _i, _i, _f, _f, ctypes.POINTER(Options), _vp, _vp, _vp]),
        "bilateral_shiftable_backward": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _f, _f, ctypes.POINTER(Options),
                                              _vp, _vp, _vp]),
        "bilateral_shiftable_train_stack": (_i, [_vp, _i, _i, _i, _i, _f, _f, ctypes.POINTER(Options), _vp, _vp,
                                                 _vp]),
        "bilateral_shiftable_backward_stack": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _f, _f,
                                                    ctypes.POINTER(Options), _vp, _vp, _vp]),
        "bilateral_shiftable_batched": (_i, [ctypes.POINTER(ImageDesc), _i, _f, ctypes.POINTER(Options), _vp]),
        "bilateral_shiftable_batched_graph": (_i, [ctypes.POINTER(ImageDesc), _i, _f, ctypes.POINTER(Options),
                                                   _i, _vp]),
        "bsk_order_for": (_i, [_f, _f]),
        "bsk_plan_info": (_i, [_i, _d, ctypes.POINTER(_i), ctypes.POINTER(_d)]),
        "bsk_truncation_error": (_d, [_i, _d]),
        "bsk_poly_order_for": (_i, [_f, _f]),
        "bsk_poly_plan_info": (_i, [_i, _f, _f, _d, ctypes.POINTER(_i), ctypes.POINTER(_d)]),
        "bsk_autotune": (_i, [_vp, _i, _i, _i, _f, _f, _vp, ctypes.POINTER(Options), ctypes.c_char_p, _vp,
                              ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_d)]),
        "bsk_batched_shape": (_i, [ctypes.POINTER(ImageDesc), _i, _f, ctypes.POINTER(Options), ctypes.POINTER(_i),
                                   ctypes.POINTER(_i), ctypes.POINTER(_i)]),
        "bsk_autotune_batched": (_i, [ctypes.POINTER(ImageDesc), _i, _f, ctypes.POINTER(Options), ctypes.c_char_p,
                                      _vp, ctypes.POINTER(_i), ctypes.POINTER(_d)]),
        "bsk_tune_cache_load": (_i, [ctypes.c_char_p]),
        "bsk_tune_cache_save": (_i, [ctypes.c_char_p]),
        "bsk_tune_cache_clear": (_i, []),
        "bsk_set_workspace_limit": (_i, [ctypes.c_longlong]),
        "bsk_last_error": (ctypes.c_char_p, []),
        "bsk_release": (_i, []),
        "bsk_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int):
    if code != BSK_OK:
        msg = load().bsk_last_error().decode(errors="replace")
        raise BskError(code, msg)
