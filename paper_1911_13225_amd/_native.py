"""ctypes declarations of the C ABI in include/dist.h.

PyTorch is imported before the library is loaded so that both share one HIP
runtime (the library then binds to the runtime PyTorch already loaded).
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime first)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdist.so")

DIST_OK, DIST_PENDING = 0, 1
ERRORS = {-1: "DIST_EINVAL", -2: "DIST_ENOMEM", -3: "DIST_EBUSY", -4: "DIST_ENOTFOUND",
          -5: "DIST_ECANCELLED", -6: "DIST_EHIP", -7: "DIST_ENUMERIC"}
ACTIVE, HIT, MISS, ESCAPED, UNCONVERGED, ERROR = 0, 1, 2, 3, 4, 5
DIST_ENUMERIC = -7
FP32, BF16 = 0, 1
REQ_RENDER, REQ_ZOPT = 0, 1


class DistError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class dist_camera(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R_wc", ctypes.c_float * 9), ("c", ctypes.c_float * 3), ("H", ctypes.c_int32), ("W", ctypes.c_int32)]


class dist_trace_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("eps", ctypes.c_float), ("normal_delta", ctypes.c_float),
                ("near_", ctypes.c_float), ("far_", ctypes.c_float), ("max_steps", ctypes.c_int32),
                ("c2f_levels", ctypes.c_int32), ("k_samples", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("want_normals", ctypes.c_int32), ("keep_history", ctypes.c_int32)]


class dist_decoder_desc(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("latent_dim", ctypes.c_int32), ("skip_layer", ctypes.c_int32),
                ("out_dims", ctypes.POINTER(ctypes.c_int32))]


class dist_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_views", ctypes.c_int32), ("cams", ctypes.POINTER(dist_camera)),
                ("prm", dist_trace_params), ("z", ctypes.c_void_p), ("depth", ctypes.c_void_p),
                ("sil", ctypes.c_void_p), ("normal", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("target_depth", ctypes.c_void_p), ("target_sil", ctypes.c_void_p), ("iters", ctypes.c_int32),
                ("lr", ctypes.c_float), ("w_depth", ctypes.c_float), ("w_sil", ctypes.c_float),
                ("z_out", ctypes.c_void_p)]


class dist_kernel_time(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("rows", ctypes.c_int64)]


class dist_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("latency_ns", ctypes.c_int64), ("queries", ctypes.c_int64),
                ("final_loss", ctypes.c_float)]


# (name, restype, argtypes)
_P = ctypes.c_void_p
_SIGS = [
    ("dist_create", ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(dist_decoder_desc), ctypes.POINTER(_P),
                                   ctypes.POINTER(_P), ctypes.c_size_t, _P]),
    ("dist_set_weights", ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _P]),
    ("dist_destroy", ctypes.c_int, [_P]),
    ("dist_render_fwd", ctypes.c_int, [_P, ctypes.POINTER(dist_camera), ctypes.c_int32, _P, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                       ctypes.POINTER(dist_trace_params), _P, _P, _P, _P, _P, _P, _P,
                                       ctypes.POINTER(_P), _P]),
    ("dist_render_bwd", ctypes.c_int, [_P, _P, _P, _P, _P, _P, ctypes.POINTER(_P), ctypes.POINTER(_P), _P]),
    ("dist_render_bwd_camera", ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    ("dist_render_bwd_implicit", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    ("dist_render_bwd_unrolled", ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    ("dist_render_color", ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    ("dist_render_color_bwd", ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]),
    ("dist_photometric_loss", ctypes.c_int, [ctypes.POINTER(dist_camera), ctypes.c_int32, _P, _P,
                                             ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_float, _P, _P,
                                             _P, _P]),
    ("dist_render_loss", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P, _P,
                                        ctypes.c_float, ctypes.c_float, ctypes.c_float, _P, _P, _P, _P, _P]),
    ("dist_adam_step", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_int32, _P]),
    ("dist_eps_for_camera", ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                           ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    ("dist_saved_free", ctypes.c_int, [_P]),
    ("dist_sdf_eval", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P, _P]),
    ("dist_sdf_eval_noalloc", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P,
                                             _P]),
    ("dist_sdf_vjp", ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P,
                                    ctypes.POINTER(_P), ctypes.POINTER(_P), _P]),
    ("dist_submit", ctypes.c_int, [_P, ctypes.POINTER(dist_request), ctypes.POINTER(ctypes.c_uint64)]),
    ("dist_poll", ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(dist_result), ctypes.c_int64]),
    ("dist_timing_enable", ctypes.c_int, [_P, ctypes.c_int]),
    ("dist_timing_read", ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(dist_kernel_time)]),
    ("dist_last_error", ctypes.c_char_p, []),
    ("dist_version", ctypes.c_char_p, []),
]
EXPORTS = [s[0] for s in _SIGS]

_lib = None


def load(path: str = LIB_PATH):
    """Load libdist.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1911_13225_amd.build`")
    lib = ctypes.CDLL(path)
    for name, res, args in _SIGS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc < 0:
        msg = _lib.dist_last_error().decode() if _lib is not None else ""
        raise DistError(rc, msg)
    return rc
