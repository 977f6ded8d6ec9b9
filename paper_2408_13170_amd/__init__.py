"""MI355X-native semi-coherent search statistic (arXiv:2408.13170).

The computation lives in libscs.so (HIP kernels for gfx950, C ABI in
include/scs.h).  This package is the thin Python binding: `_binding` mirrors
the C entry points one to one, `Context` bundles one search's handle.
"""
from __future__ import annotations

from . import _binding as B
from ._binding import (SCS_MAX_SEGMENTS, SCS_MEM_DEVICE, SCS_MEM_HOST, SCS_PREC_FP64, SCS_PREC_MIXED,
                       SCS_RESP_LISA_FD_AE, SCS_RESP_LISA_LF_AE, SCS_RESP_NONE, SCS_SEG_EQUAL_SNR, SCS_SEG_EXPLICIT,
                       SCS_SEG_UNIFORM, SCS_SUPPORT_FULL, SCS_SUPPORT_TOBS, ScsError)

__all__ = ["B", "Context", "ScsError", "SCS_PREC_FP64", "SCS_PREC_MIXED", "SCS_RESP_NONE", "SCS_RESP_LISA_LF_AE",
           "SCS_RESP_LISA_FD_AE", "SCS_SUPPORT_FULL", "SCS_SUPPORT_TOBS", "SCS_SEG_EQUAL_SNR", "SCS_SEG_UNIFORM",
           "SCS_SEG_EXPLICIT", "SCS_MAX_SEGMENTS", "SCS_MEM_HOST", "SCS_MEM_DEVICE"]


class Context:
    """One search: data + PSD on the device, model, segmentation."""

    def __init__(self, device=0):
        self.h = B.scs_ctx_create(device)
        self.N = 1

    def close(self):
        if self.h is not None:
            B.scs_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_data(self, d_ri, psd, f_min, df):
        B.scs_load_data(self.h, d_ri, psd, f_min, df)
        return self

    def set_model(self, pn_order, response, support, t_obs=0.0, block_len=0, orbit_phase0=0.0,
                  cartwheel_phase0=0.0):
        B.scs_set_model(self.h, pn_order, response, support, t_obs, block_len, orbit_phase0, cartwheel_phase0)
        return self

    def define_segmentation(self, N, mode=SCS_SEG_EQUAL_SNR, G=1024, edges=None):
        B.scs_define_segmentation(self.h, N, mode, G, edges)
        self.N = N
        return self

    def evaluate(self, theta, ups, prec=SCS_PREC_FP64, seg=None, stream=None):
        B.scs_evaluate(self.h, theta, ups, prec, seg, stream)
        return ups

    def bounds(self, P):
        return B.scs_last_bounds(self.h, P, self.N)

    def waveform(self, theta, h_ri, stream=None):
        B.scs_waveform(self.h, theta, h_ri, stream)
        return h_ri

    def stats(self, reset=False):
        return B.scs_ctx_stats(self.h, reset)

    def footprint(self, P, N, prec=SCS_PREC_FP64):
        return B.scs_footprint(self.h, P, N, prec)
