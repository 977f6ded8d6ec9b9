"""MI355X-native semi-coherent search statistic (arXiv:2408.13170).

The computation lives in libscs.so (HIP kernels for gfx950, C ABI in
include/scs.h).  This package is the thin Python binding: `_binding` mirrors
the C entry points one to one.
"""
from __future__ import annotations

from . import _binding as B
from ._binding import (SCS_MAX_SEGMENTS, SCS_MEM_DEVICE, SCS_MEM_HOST, SCS_PREC_FP64, SCS_PREC_MIXED,
                       SCS_RESP_LISA_FD_AE, SCS_RESP_LISA_LF_AE, SCS_RESP_NONE, SCS_SEG_EQUAL_SNR, SCS_SEG_EXPLICIT,
                       SCS_SEG_UNIFORM, SCS_SUPPORT_FULL, SCS_SUPPORT_TOBS, ScsError)

__all__ = ["B", "ScsError", "SCS_PREC_FP64", "SCS_PREC_MIXED", "SCS_RESP_NONE", "SCS_RESP_LISA_LF_AE",
           "SCS_RESP_LISA_FD_AE", "SCS_SUPPORT_FULL", "SCS_SUPPORT_TOBS", "SCS_SEG_EQUAL_SNR", "SCS_SEG_UNIFORM",
           "SCS_SEG_EXPLICIT", "SCS_MAX_SEGMENTS", "SCS_MEM_HOST", "SCS_MEM_DEVICE"]
