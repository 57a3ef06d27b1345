"""ctypes loader for libadjwave.so (the C ABI in include/adjwave.h).

Loading fails loudly: there is no CPU fallback. Build the library first with
``python -m paper_1707_02018_amd.build``.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadjwave.so")

MAX_TAPS = 16
MAX_LEVELS = 8
MAX_RADIUS = 12

OK, EINVAL, EUNSUPPORTED, EHIP = 0, -1, -2, -3
F32, F64 = 0, 1
BC = {"zpd": 0, "sym": 1, "per": 2, "per_ext": 3}


class Wavelet(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("filter_len", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("lo", ctypes.c_double * MAX_TAPS), ("biorthogonal", ctypes.c_int32),
                ("lo_analysis", ctypes.c_double * MAX_TAPS)]


class Blur(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("taps", ctypes.c_double * (2 * MAX_RADIUS + 1))]


class FistaState(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("resid", ctypes.c_void_p),
                ("obj", ctypes.c_void_p), ("k", ctypes.c_int64), ("t", ctypes.c_double),
                ("gradient", ctypes.c_int32)]


_P = ctypes.c_void_p
_W = ctypes.POINTER(Wavelet)
_B = ctypes.POINTER(Blur)
_i32, _i64, _dbl, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t

# name -> (argtypes); every entry point returns aw_status (int) except aw_last_error
SIGNATURES = {
    "aw_daubechies": [_i32, ctypes.POINTER(_dbl)],
    "aw_cdf97": [ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)],
    "aw_gaussian_psf": [_dbl, _i32, ctypes.POINTER(_dbl)],
    "aw_wavelet_layout": [_W, ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "aw_workspace_size": [_W, _B, _i32, _i32, ctypes.POINTER(_sz)],
    "wavelet_synth": [_W, _i32, _i32, _P, _P, _P, _sz, _P],
    "wavelet_synth_adjoint": [_W, _i32, _i32, _P, _P, _P, _sz, _P],
    "aw_wavelet_analysis": [_W, _i32, _i32, _P, _P, _P, _sz, _P],
    "aw_wavelet_analysis_adjoint": [_W, _i32, _i32, _P, _P, _P, _sz, _P],
    "blur": [_B, _i32, _i32, _P, _P, _P],
    "blur_adjoint": [_B, _i32, _i32, _P, _P, _P],
    "aw_apply_A": [_W, _B, _i32, _i32, _P, _P, _P, _sz, _P],
    "aw_apply_A_fused": [_W, _B, _i32, _i32, _P, _P, _P, _P, _sz, _P],
    "aw_apply_A_adjoint": [_W, _B, _i32, _i32, _P, _P, _P, _sz, _P],
    "aw_apply_A_adjoint_fused": [_W, _B, _i32, _i32, _P, _P, _P, _sz, _P],
    "fista_step": [_W, _B, _i32, _i32, _P, _dbl, _dbl, ctypes.POINTER(FistaState), _i32, _P, _sz,
                   _P],
    "fista_step_noalloc": [_W, _B, _i32, _i32, _P, _dbl, _dbl, ctypes.POINTER(FistaState), _i32,
                           _P],
    "aw_fista_update": [_W, _i32, _i32, _P, _dbl, _dbl, ctypes.POINTER(FistaState), _i32, _P, _sz,
                        _P],
    "aw_objective": [_W, _B, _i32, _i32, _P, _dbl, _P, _P, _P, _sz, _P],
    "conv_adjoint_pair": [_i32, _i32, _i32, _i32, _P, _P, _P, _P, _P, _P, _P],
    "aw_blur_dct_create": [_i32, _i32, _i32, ctypes.POINTER(_dbl), _i32, ctypes.POINTER(_P)],
    "aw_blur_dct_destroy": [_P],
    "aw_blur_dct_workspace": [_P, _i32, ctypes.POINTER(_sz)],
    "aw_blur_dct_apply": [_P, _i32, _P, _P, _P, _sz, _P],
    "aw_conv_multichannel": [_i32, _i32, _i32, _i32, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "aw_huber_tv": [_i32, _i32, _i32, _P, _dbl, _dbl, _P, _P, _P],
    "aw_prox_l1": [_i32, _i64, _P, _P, _dbl, _dbl, _P, _P, _P],
    "aw_batch_create": [_i32, _W, _B, ctypes.POINTER(_P)],
    "aw_batch_destroy": [_P],
    "aw_batch_layout": [_P, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_sz)],
    "aw_batch_set_config": [_P, ctypes.POINTER(_i32)],
    "aw_batch_bind": [_P, _P, _P, _P, _P, _sz, _dbl, _dbl],
    "aw_batch_control": [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P)],
    "aw_batch_reset": [_P, _P],
    "aw_batch_step": [_P, _P],
    "aw_cnn_sizes": [_i32, _i32, _i32, ctypes.POINTER(_sz), ctypes.POINTER(_sz),
                     ctypes.POINTER(_sz)],
    "aw_cnn_pack": [_P, _P, _P],
    "aw_cnn_forward": [_P, _i32, _i32, _i32, _P, _P, _P, _P],
    "aw_cnn_backward": [_P, _i32, _i32, _i32, _P, _P, _P, _P, _P, _P, _sz, _P],
    "aw_adam_step": [_P, _P, _P, _P, _i64, _i32, _dbl, _dbl, _dbl, _dbl, _P],
    "aw_sq_error": [_i64, _P, _P, _dbl, _P, _P, _P, _sz, _P],
    "aw_sq_error_workspace": [_i64, ctypes.POINTER(_sz)],
    "aw_soft_threshold": [_i64, _P, _dbl, _P, _P],
}

_lib = None


def load() -> ctypes.CDLL:
    """Load (once) and type the shared library; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1707_02018_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.aw_last_error.restype = ctypes.c_char_p
    lib.aw_last_error.argtypes = []
    lib.aw_batch_last_error.restype = ctypes.c_char_p
    lib.aw_batch_last_error.argtypes = []
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    _lib = lib
    return lib


class AdjwaveError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed (status {status}): {msg}")
        self.status = status


def check(fn: str, status: int) -> None:
    if status != OK:
        lib = load()
        msg = (lib.aw_batch_last_error() if fn.startswith("aw_batch") else lib.aw_last_error())
        raise AdjwaveError(fn, status, msg.decode())
