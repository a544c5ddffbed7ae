"""ctypes declarations of the hsbuild C-ABI (include/hsbuild.h).

Loads paper_1712_07206_amd/libhsbuild.so.  There is no fallback: if the
library is missing, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhsbuild.so")

HSB_OK = 0
HSB_ERR_ARG = -1
HSB_ERR_SHAPE = -2
HSB_ERR_WORKSPACE = -3
HSB_ERR_DEVICE = -4
HSB_ERR_UNSUPPORTED = -5
HSB_ERR_NUMERIC = -6
STATUS_NAMES = {0: "HSB_OK", -1: "HSB_ERR_ARG", -2: "HSB_ERR_SHAPE", -3: "HSB_ERR_WORKSPACE",
                -4: "HSB_ERR_DEVICE", -5: "HSB_ERR_UNSUPPORTED", -6: "HSB_ERR_NUMERIC"}

HSB_FP64 = 0
HSB_SPLIT_FP16 = 1
HSB_SPLIT_BF16 = 2
HSB_SPLIT_INT8 = 3
HSB_SPLIT_CRT = 4
HSB_SPLIT_CRT_BF16 = 5
HSB_SPLIT_CRT_FP16 = 6
HSB_PROBE_FP64 = 0
HSB_PROBE_INT8 = 1
HSB_PROBE_INT8_RANDOM = 2

HSB_MODE_FORWARD = 0
HSB_MODE_BACKWARD = 1
HSB_MODE_BATCH = 2
HSB_MODE_COEFFICIENTS = 3
HSB_MODE_FACTORED = 4
HSB_MODE_HSDLA = 5
HSB_MODE_REAL = 6
HSB_MODE_EIGEN = 7

EXPORTS = ("hsbuild_create", "hsbuild_destroy", "hsbuild_workspace_bytes", "hsbuild_coefficients",
           "hsbuild_forward", "hsbuild_forward_factored", "hsbuild_forward_hsdla", "hsbuild_forward_real", "hsbuild_eigensolve",
           "hsbuild_forward_coefficients",
           "hsbuild_backward",
           "hsbuild_batch", "hsbuild_last_error",
           "hsbuild_host_bessel", "hsbuild_host_angular", "hsbuild_set_timing", "hsbuild_stage_times",
           "hsbuild_set_option", "hsbuild_get_option", "hsbuild_mfma_probe", "hsbuild_forward_static")

HSB_STATIC_SCRATCH_BYTES = 256 << 20

HSB_OPT_TILE_GROUP = 1
HSB_OPT_HS_WAVES = 2
HSB_OPT_SPLIT_K = 3
HSB_TIMING_STAGES = 4


class HsbConfig(ctypes.Structure):
    _fields_ = [
        ("n_types", c_int32), ("n_atoms", c_int32), ("l_max", c_int32), ("max_ng", c_int32),
        ("lattice", c_double * 9),
        ("atom_type", POINTER(c_int32)), ("r_mt", POINTER(c_double)),
        ("radial", POINTER(c_double)), ("udot_norm2", POINTER(c_double)),
        ("precision", c_int32), ("n_slices", c_int32),
    ]


class HSBuildError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), message))
        self.code = code


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhsbuild.so is not built (%s); run __graft_entry__.build() or "
                          "python -m paper_1712_07206_amd.build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    L.hsbuild_create.argtypes = [POINTER(HsbConfig), POINTER(c_void_p)]
    L.hsbuild_create.restype = c_int
    L.hsbuild_destroy.argtypes = [c_void_p]
    L.hsbuild_destroy.restype = None
    L.hsbuild_workspace_bytes.argtypes = [c_void_p, c_int32, c_int32, POINTER(c_int32)]
    L.hsbuild_workspace_bytes.restype = c_size_t
    L.hsbuild_coefficients.argtypes = [c_void_p, POINTER(c_double), c_int32, c_void_p, c_void_p, c_void_p,
                                       c_void_p, c_size_t, c_void_p]
    L.hsbuild_coefficients.restype = c_int
    L.hsbuild_forward.argtypes = [c_void_p, POINTER(c_double), c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_size_t, c_void_p]
    L.hsbuild_forward.restype = c_int
    L.hsbuild_forward_static.argtypes = [c_void_p, POINTER(c_double), c_int32, c_void_p, c_void_p, c_void_p,
                                         c_void_p, c_void_p, c_void_p]
    L.hsbuild_forward_static.restype = c_int
    L.hsbuild_forward_factored.argtypes = [c_void_p, POINTER(c_double), c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_size_t, c_void_p]
    L.hsbuild_forward_factored.restype = c_int
    L.hsbuild_forward_hsdla.argtypes = [c_void_p, c_int32, POINTER(c_double), c_int32, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.hsbuild_forward_hsdla.restype = c_int
    L.hsbuild_forward_real.argtypes = [c_void_p, POINTER(c_double), c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.hsbuild_forward_real.restype = c_int
    L.hsbuild_eigensolve.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
                                     c_size_t, c_void_p]
    L.hsbuild_eigensolve.restype = c_int
    L.hsbuild_forward_coefficients.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                               c_size_t, c_void_p]
    L.hsbuild_forward_coefficients.restype = c_int
    L.hsbuild_backward.argtypes = [c_void_p, POINTER(c_double), c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.hsbuild_backward.restype = c_int
    L.hsbuild_batch.argtypes = [c_void_p, c_int32, POINTER(c_double), POINTER(c_int32), c_void_p,
                                POINTER(c_int64), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                c_void_p]
    L.hsbuild_batch.restype = c_int
    L.hsbuild_last_error.argtypes = [c_void_p]
    L.hsbuild_last_error.restype = c_char_p
    L.hsbuild_host_bessel.argtypes = [c_int32, c_double, POINTER(c_double), POINTER(c_double)]
    L.hsbuild_host_bessel.restype = c_int
    L.hsbuild_host_angular.argtypes = [c_int32, POINTER(c_double), c_double, c_void_p]
    L.hsbuild_host_angular.restype = c_int
    L.hsbuild_set_timing.argtypes = [c_void_p, c_int32]
    L.hsbuild_set_timing.restype = c_int
    L.hsbuild_stage_times.argtypes = [c_void_p, POINTER(c_double), POINTER(c_int32)]
    L.hsbuild_stage_times.restype = c_int
    L.hsbuild_mfma_probe.argtypes = [c_int32, c_int32, c_int32, c_void_p, c_size_t, c_void_p, POINTER(c_double)]
    L.hsbuild_mfma_probe.restype = c_int
    L.hsbuild_set_option.argtypes = [c_void_p, c_int32, c_int32]
    L.hsbuild_set_option.restype = c_int
    L.hsbuild_get_option.argtypes = [c_void_p, c_int32, POINTER(c_int32)]
    L.hsbuild_get_option.restype = c_int
    _lib = L
    return L


def last_error(handle) -> str:
    msg = lib().hsbuild_last_error(handle)
    return msg.decode() if msg else ""


def check(code: int, handle) -> None:
    if code != HSB_OK:
        raise HSBuildError(code, last_error(handle))
