"""MI355X-native builder of the FLAPW muffin-tin Hamiltonian and overlap matrices.

The computation lives in libhsbuild.so (HIP, gfx950) behind the C-ABI of
include/hsbuild.h; this package holds its sources (csrc/), the build script
and a thin ctypes/PyTorch binding.
"""
from . import _native
from ._native import (HSBuildError, HSB_FP64, HSB_SPLIT_FP16, HSB_SPLIT_BF16, HSB_SPLIT_INT8, HSB_SPLIT_CRT,
                      HSB_SPLIT_CRT_BF16, HSB_SPLIT_CRT_FP16)

__all__ = ["_native", "HSBuildError", "HSB_FP64", "HSB_SPLIT_FP16", "HSB_SPLIT_BF16", "HSB_SPLIT_INT8",
           "HSB_SPLIT_CRT", "HSB_SPLIT_CRT_BF16", "HSB_SPLIT_CRT_FP16"]
