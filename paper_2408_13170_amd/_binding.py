"""ctypes binding of libscs (include/scs.h).  Argument marshalling only: every
step of the statistic runs in the HIP kernels of libscs.so.

Functions keep the C names.  Pointer arguments accept numpy arrays (host) or
torch CUDA tensors (device); the binding passes raw pointers and the memory
kind, and raises ScsError with scs_last_error() on a negative return code.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libscs.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "scs.h")

SCS_OK, SCS_EINVAL, SCS_ENOMEM, SCS_EDEVICE, SCS_EBUSY, SCS_ESTATE = 0, -1, -2, -3, -4, -5
SCS_MEM_HOST, SCS_MEM_DEVICE = 0, 1
SCS_PREC_FP64, SCS_PREC_MIXED = 0, 1
SCS_RESP_NONE, SCS_RESP_LISA_LF_AE, SCS_RESP_LISA_FD_AE = 0, 1, 2
SCS_SUPPORT_FULL, SCS_SUPPORT_TOBS = 0, 1
SCS_SEG_EQUAL_SNR, SCS_SEG_UNIFORM, SCS_SEG_EXPLICIT = 0, 1, 2
SCS_MAX_SEGMENTS = 1 << 20


class ScsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libscs error {code}: {msg}")
        self.code = code


class scs_model(C.Structure):
    _fields_ = [("pn_order", C.c_int32), ("response", C.c_int32), ("support", C.c_int32),
                ("block_len", C.c_int32), ("t_obs", C.c_double), ("orbit_phase0", C.c_double),
                ("cartwheel_phase0", C.c_double), ("eccentric", C.c_int32), ("sparse_stride", C.c_int32)]


class scs_batch_item(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("N", C.c_int32), ("pad", C.c_int32), ("P", C.c_int64),
                ("theta", C.c_void_p), ("ups", C.c_void_p), ("seg", C.c_void_p)]


class scs_request_done(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int32), ("pad", C.c_int32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_launch", C.c_double), ("t_done", C.c_double)]


class scs_server_counters(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64), ("launches", C.c_int64),
                ("max_batch", C.c_int64), ("max_inflight", C.c_int64), ("hbm_in_use", C.c_uint64),
                ("hbm_peak", C.c_uint64)]


class scs_pso_params(C.Structure):
    _fields_ = [("omega", C.c_double), ("phi_p", C.c_double), ("phi_g", C.c_double),
                ("eps", C.c_double * 8)]


class scs_search_params(C.Structure):
    _fields_ = [("n_swarms", C.c_int32), ("G", C.c_int32), ("particles", C.c_int64), ("conv_tol", C.c_double),
                ("conv_window", C.c_int32), ("kmeans_iters", C.c_int32), ("prec", C.c_int32), ("pad", C.c_int32),
                ("seed", C.c_uint64)]


class scs_rung(C.Structure):
    _fields_ = [("N", C.c_int32), ("max_iters", C.c_int32), ("prm", scs_pso_params)]


class scs_rung_report(C.Structure):
    _fields_ = [("N", C.c_int32), ("n_swarms", C.c_int32), ("iterations", C.c_int32), ("converged", C.c_int32),
                ("best_val", C.c_double), ("seconds", C.c_double)]


_lib = None

_SIGS = {
    "scs_ctx_create": [C.POINTER(C.c_void_p), C.c_int],
    "scs_ctx_destroy": [C.c_void_p],
    "scs_load_data": [C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_int32],
    "scs_set_model": [C.c_void_p, C.POINTER(scs_model)],
    "scs_define_segmentation": [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p],
    "scs_evaluate": [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
    "scs_evaluate_noalloc": [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p],
    "scs_last_bounds": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p],
    "scs_evaluate_stats": [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p],
    "scs_data_norm": [C.c_void_p, C.POINTER(C.c_double)],
    "scs_make_realisations": [C.c_void_p, C.c_int64, C.c_uint64, C.c_int64, C.c_double, C.c_void_p, C.c_void_p],
    "scs_evaluate_streams": [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p],
    "scs_loglike": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                    C.c_void_p],
    "scs_waveform": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
    "scs_ctx_stats": [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int32],
    "scs_ctx_profile": [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)],
    "scs_footprint": [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)],
    "scs_evaluate_batched": [C.POINTER(scs_batch_item), C.c_int32, C.c_int32, C.c_void_p],
    "scs_graph_create": [C.POINTER(C.c_void_p), C.POINTER(scs_batch_item), C.c_int32, C.c_int32],
    "scs_graph_launch": [C.c_void_p, C.c_void_p],
    "scs_graph_destroy": [C.c_void_p],
    "scs_autotune": [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_int32, C.c_char_p],
    "scs_swarm_create": [C.c_void_p, C.POINTER(C.c_void_p), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                         C.c_uint64, C.c_uint32],
    "scs_swarm_destroy": [C.c_void_p],
    "scs_pso_step": [C.c_void_p, C.POINTER(scs_pso_params), C.c_int32, C.c_void_p],
    "scs_pso_step_swarms": [C.c_void_p, C.c_int32, C.POINTER(scs_pso_params), C.c_int32, C.c_void_p, C.c_void_p],
    "scs_swarm_read": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                       C.POINTER(C.c_double), C.POINTER(C.c_uint32)],
    "scs_swarm_write": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                        C.c_uint32],
    "scs_swarm_device_ptrs": [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)],
    "scs_pso_move": [C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                     C.POINTER(scs_pso_params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32,
                     C.c_uint32, C.c_void_p],
    "scs_pso_best": [C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "scs_theta_dim": [C.c_void_p, C.POINTER(C.c_int32)],
    "scs_peak_probe": [C.c_int32, C.POINTER(C.c_double)],
    "scs_autotune_batch": [C.POINTER(scs_batch_item), C.c_int32, C.c_int32, C.c_char_p],
    "scs_distance_amplitude": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
    "scs_ctx_info": [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                     C.POINTER(C.c_int64)],
    "scs_server_create": [C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.c_uint64, C.c_int32],
    "scs_server_submit": [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p,
                          C.POINTER(C.c_uint64)],
    "scs_server_poll": [C.c_void_p, C.POINTER(scs_request_done), C.c_int32, C.c_int32, C.POINTER(C.c_int32)],
    "scs_server_stats": [C.c_void_p, C.POINTER(scs_server_counters)],
    "scs_server_clock": [C.c_void_p],
    "scs_server_destroy": [C.c_void_p],
    "scs_search_create": [C.c_void_p, C.POINTER(scs_search_params), C.c_void_p, C.c_void_p, C.c_void_p,
                          C.POINTER(C.c_void_p)],
    "scs_search_run_rung": [C.c_void_p, C.POINTER(scs_rung), C.POINTER(scs_rung_report), C.c_void_p],
    "scs_search_swarms": [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p, C.c_void_p],
    "scs_search_destroy": [C.c_void_p],
    "scs_kmeans": [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_void_p, C.c_void_p,
                   C.POINTER(C.c_int32)],
    "scs_kmeans_device": [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_void_p,
                          C.c_void_p, C.POINTER(C.c_int32), C.c_void_p],
    "scs_last_error": [],
}
_RESTYPES = {"scs_last_error": C.c_char_p, "scs_server_clock": C.c_double}


def lib():
    """Load libscs.so from the package directory (fails loudly if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: build it with paper_2408_13170_amd/build.py "
                              "(or __graft_entry__.build())")
        L = C.CDLL(LIBPATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _RESTYPES.get(name, C.c_int)
        _lib = L
    return _lib


def header_symbols():
    """Names of every function declared in include/scs.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|double|const char\*)\s+(scs_\w+)\s*\(", txt, re.M)))


def _check(rc):
    if rc != 0:
        msg = lib().scs_last_error()
        raise ScsError(rc, msg.decode() if msg else "")


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def ptr(x):
    """Raw pointer and memory kind of a numpy array or torch tensor (or None)."""
    if x is None:
        return None, None
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(x.data_ptr()), (SCS_MEM_DEVICE if x.is_cuda else SCS_MEM_HOST)
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return C.c_void_p(x.ctypes.data), SCS_MEM_HOST
    raise TypeError(f"unsupported buffer type {type(x)}")


# ---- argument checks: the kernels index these buffers by the shapes below,
# so a wrong dtype, width or length is refused here, before any call into the
# library (a raw pointer carries no size for the library to check).
def _is_f64(x):
    if _is_torch(x):
        import torch

        return x.dtype == torch.float64
    return isinstance(x, np.ndarray) and x.dtype == np.float64


def need_f64(x, name, shape):
    """x must be a float64 buffer of exactly this shape (None entries: any)."""
    if x is None:
        raise ValueError(f"{name} is missing")
    if not _is_f64(x):
        raise ValueError(f"{name} must be float64, got {getattr(x, 'dtype', type(x))}")
    got = tuple(x.shape)
    if len(got) != len(shape) or any(w is not None and g != w for g, w in zip(got, shape)):
        want = tuple("*" if w is None else w for w in shape)
        raise ValueError(f"{name} must have shape {want}, got {got}")


def _same_kind(*pairs):
    kinds = {k for _, k in pairs if k is not None}
    if len(kinds) > 1:
        raise ValueError("all buffers of a call must live in the same memory (host or device)")
    return kinds.pop() if kinds else None


def scs_ctx_info(ctx):
    """{'theta_dim', 'N', 'n_chan', 'K'} of a context."""
    d, n, c, k = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
    _check(lib().scs_ctx_info(ctx, C.byref(d), C.byref(n), C.byref(c), C.byref(k)))
    return {"theta_dim": d.value, "N": n.value, "n_chan": c.value, "K": k.value}


def check_eval_args(theta, ups, seg, dim, N, name_out="ups", width=1):
    """theta [P, dim]; out [P] (width 1) or [P, width]; seg [P, N, 3] or None."""
    need_f64(theta, "theta", (None, dim))
    P = theta.shape[0]
    need_f64(ups, name_out, (P,) if width == 1 else (P, width))
    if seg is not None:
        need_f64(seg, "seg", (P, N, 3))
    return P


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def current_stream():
    import torch

    return torch.cuda.current_stream()


# ---------------------------------------------------------------- wrappers
def scs_ctx_create(device=0):
    h = C.c_void_p()
    _check(lib().scs_ctx_create(C.byref(h), device))
    return h


def scs_ctx_destroy(ctx):
    _check(lib().scs_ctx_destroy(ctx))


def scs_load_data(ctx, d_ri, psd, f_min, df):
    """d_ri [n_chan, K, 2] and psd [n_chan, K] (float64, host or device)."""
    need_f64(psd, "psd", (None, None))
    n_chan, K = psd.shape[0], psd.shape[1]
    need_f64(d_ri, "d_ri", (n_chan, K, 2))
    pd, kd = ptr(d_ri)
    pp, kp = ptr(psd)
    if kd != kp:
        raise ValueError("data and psd must live in the same memory")
    _check(lib().scs_load_data(ctx, n_chan, K, f_min, df, pd, pp, kd))


def scs_set_model(ctx, pn_order, response, support, t_obs=0.0, block_len=0, orbit_phase0=0.0,
                  cartwheel_phase0=0.0, eccentric=0, sparse_stride=0):
    m = scs_model(pn_order, response, support, block_len, t_obs, orbit_phase0, cartwheel_phase0, eccentric,
                  sparse_stride)
    _check(lib().scs_set_model(ctx, C.byref(m)))


def scs_define_segmentation(ctx, N, mode=SCS_SEG_EQUAL_SNR, G=1024, edges=None):
    e = None
    if edges is not None:
        edges = np.ascontiguousarray(edges, dtype=np.int64)
        e = C.c_void_p(edges.ctypes.data)
    _check(lib().scs_define_segmentation(ctx, N, mode, G, e))


def scs_evaluate(ctx, theta, ups, prec=SCS_PREC_FP64, seg=None, stream=None):
    """theta [P,D] -> ups [P] (and seg [P,N,3]); all numpy or all CUDA tensors."""
    info = scs_ctx_info(ctx)
    P = check_eval_args(theta, ups, seg, info["theta_dim"], info["N"])
    pt, kt = ptr(theta)
    pu, ku = ptr(ups)
    ps, ks = ptr(seg)
    if kt != ku or (seg is not None and ks != kt):
        raise ValueError("theta, ups and seg must live in the same memory")
    if kt == SCS_MEM_DEVICE and stream is None:
        stream = current_stream()
    _check(lib().scs_evaluate(ctx, P, pt, prec, pu, ps, kt, _stream(stream)))


def scs_evaluate_noalloc(ctx, theta, ups, prec=SCS_PREC_FP64, seg=None, stream=None):
    """scs_evaluate without any allocation: theta [P,D] -> ups [P] (and seg
    [P,N,3]), CUDA tensors only; buffers live in the library's static device
    scratch of SCS_NOALLOC_SCRATCH_BYTES."""
    info = scs_ctx_info(ctx)
    P = check_eval_args(theta, ups, seg, info["theta_dim"], info["N"])
    pt, kt = ptr(theta)
    pu, ku = ptr(ups)
    ps, ks = ptr(seg)
    if kt != SCS_MEM_DEVICE or ku != SCS_MEM_DEVICE or (seg is not None and ks != SCS_MEM_DEVICE):
        raise ValueError("scs_evaluate_noalloc takes device tensors only")
    if stream is None:
        stream = current_stream()
    _check(lib().scs_evaluate_noalloc(ctx, P, pt, prec, pu, ps, _stream(stream)))


SCS_NOALLOC_SCRATCH_BYTES = 64 << 20
SCS_NSTATS = 5


def scs_evaluate_stats(ctx, theta, stats, prec=SCS_PREC_FP64, stream=None):
    """theta [P,7] -> stats [P,5] = (Upsilon_N, hat O_N, <h|h>, Re <d|h>, Im <d|h>)
    for the unit-amplitude template; both numpy or both CUDA tensors."""
    info = scs_ctx_info(ctx)
    P = check_eval_args(theta, stats, None, info["theta_dim"], info["N"], "stats", SCS_NSTATS)
    pt, kt = ptr(theta)
    ps, ks = ptr(stats)
    if kt != ks:
        raise ValueError("theta and stats must live in the same memory")
    if kt == SCS_MEM_DEVICE and stream is None:
        stream = current_stream()
    _check(lib().scs_evaluate_stats(ctx, P, pt, prec, ps, kt, _stream(stream)))


def scs_data_norm(ctx):
    v = C.c_double()
    _check(lib().scs_data_norm(ctx, C.byref(v)))
    return v.value


def scs_loglike(ctx, stats, amp, phase=None, logl_semi=None, logl_coh=None, stream=None):
    """Log-likelihoods of A h e^{i phi} from scs_evaluate_stats rows into the
    given output arrays (either may be None); all arrays in one memory."""
    need_f64(stats, "stats", (None, SCS_NSTATS))
    P = stats.shape[0]
    need_f64(amp, "amp", (P,))
    for name, x in (("phase", phase), ("logl_semi", logl_semi), ("logl_coh", logl_coh)):
        if x is not None:
            need_f64(x, name, (P,))
    ptrs = [ptr(x) for x in (stats, amp, phase, logl_semi, logl_coh)]
    kinds = {k for (p, k), x in zip(ptrs, (stats, amp, phase, logl_semi, logl_coh)) if x is not None}
    if len(kinds) != 1:
        raise ValueError("stats, amp, phase and the outputs must live in the same memory")
    kind = kinds.pop()
    if kind == SCS_MEM_DEVICE and stream is None:
        stream = current_stream()
    _check(lib().scs_loglike(ctx, P, *(p for p, _ in ptrs), kind, _stream(stream)))


def scs_distance_amplitude(ctx, theta, dl_mpc, amp, stream=None):
    """Absolute template amplitude A [P] for distances dl_mpc [P] (Mpc) and the
    chirp masses of theta [P][D]; all arrays in one memory."""
    info = scs_ctx_info(ctx)
    need_f64(theta, "theta", (None, info["theta_dim"]))
    P = theta.shape[0]
    need_f64(dl_mpc, "dl_mpc", (P,))
    need_f64(amp, "amp", (P,))
    ptrs = [ptr(x) for x in (theta, dl_mpc, amp)]
    kinds = {k for _, k in ptrs}
    if len(kinds) != 1:
        raise ValueError("theta, dl_mpc and amp must live in the same memory")
    kind = kinds.pop()
    if kind == SCS_MEM_DEVICE and stream is None:
        stream = current_stream()
    _check(lib().scs_distance_amplitude(ctx, P, *(p for p, _ in ptrs), kind, _stream(stream)))


def scs_make_realisations(ctx, streams, seed, r0=0, scale=1.0, stream=None):
    """Fill the CUDA tensor streams [n_chan, K, R, 2] with scale * d + noise realisations r0 .. r0 + R - 1."""
    if not _is_torch(streams) or not streams.is_cuda:
        raise TypeError("streams must be a CUDA tensor [n_chan, K, R, 2]")
    info = scs_ctx_info(ctx)
    need_f64(streams, "streams", (info["n_chan"], info["K"], None, 2))
    R = streams.shape[2]
    p, _ = ptr(streams)
    _check(lib().scs_make_realisations(ctx, R, seed, r0, scale, p, _stream(stream or current_stream())))


def scs_evaluate_streams(ctx, theta, streams, stats, stream=None):
    """theta numpy [D] (the context's theta width); streams CUDA [n_chan, K, R, 2]; stats CUDA [R, 5] out."""
    th = np.ascontiguousarray(theta, dtype=np.float64).ravel()
    if not (_is_torch(streams) and streams.is_cuda and _is_torch(stats) and stats.is_cuda):
        raise TypeError("streams and stats must be CUDA tensors")
    info = scs_ctx_info(ctx)
    need_f64(th, "theta", (info["theta_dim"],))
    need_f64(streams, "streams", (info["n_chan"], info["K"], None, 2))
    R = streams.shape[2]
    need_f64(stats, "stats", (R, SCS_NSTATS))
    ps, _ = ptr(streams)
    pt, _ = ptr(stats)
    _check(lib().scs_evaluate_streams(ctx, C.c_void_p(th.ctypes.data), R, ps, pt, _stream(stream or current_stream())))


def scs_last_bounds(ctx, P, N):
    sup = np.empty((P, 2), dtype=np.int32)
    bnd = np.empty((P, N + 1), dtype=np.int32)
    _check(lib().scs_last_bounds(ctx, P, C.c_void_p(sup.ctypes.data), C.c_void_p(bnd.ctypes.data)))
    return sup, bnd


def scs_waveform(ctx, theta, h_ri, stream=None):
    info = scs_ctx_info(ctx)
    need_f64(theta, "theta", (info["theta_dim"],))
    need_f64(h_ri, "h_ri", (info["n_chan"], info["K"], 2))
    pt, kt = ptr(theta)
    ph, kh = ptr(h_ri)
    if kt != kh:
        raise ValueError("theta and h must live in the same memory")
    if kt == SCS_MEM_DEVICE and stream is None:
        stream = current_stream()
    _check(lib().scs_waveform(ctx, pt, ph, kt, _stream(stream)))


def scs_ctx_stats(ctx, reset=False):
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().scs_ctx_stats(ctx, C.byref(a), C.byref(b), C.byref(c), int(reset)))
    return a.value, b.value, c.value


def scs_ctx_profile(ctx, enable=-1):
    n, ms = C.c_int64(), C.c_double()
    _check(lib().scs_ctx_profile(ctx, enable, C.byref(n), C.byref(ms)))
    return n.value, ms.value


def scs_footprint(ctx, P, N, prec=SCS_PREC_FP64):
    b = C.c_size_t()
    _check(lib().scs_footprint(ctx, P, N, prec, C.byref(b)))
    return b.value


def _items(items):
    arr = (scs_batch_item * len(items))()
    for i, it in enumerate(items):
        ctx, N, theta, ups = it[:4]
        seg = it[4] if len(it) > 4 else None
        for x in (theta, ups, seg):
            if x is not None and not (_is_torch(x) and x.is_cuda and x.is_contiguous()):
                raise ValueError(f"item {i}: theta, ups and seg must be contiguous CUDA tensors")
        check_eval_args(theta, ups, seg, scs_ctx_info(ctx)["theta_dim"], N)
        arr[i] = scs_batch_item(ctx.value if isinstance(ctx, C.c_void_p) else ctx, N, 0, theta.shape[0],
                                theta.data_ptr(), ups.data_ptr(), seg.data_ptr() if seg is not None else None)
    return arr


def scs_evaluate_batched(items, prec=SCS_PREC_FP64, stream=None):
    """items: list of (ctx, N, theta_cuda [P,7], ups_cuda [P][, seg_cuda])."""
    arr = _items(items)
    if stream is None:
        stream = current_stream()
    _check(lib().scs_evaluate_batched(arr, len(items), prec, _stream(stream)))


def scs_graph_create(items, prec=SCS_PREC_FP64):
    arr = _items(items)
    h = C.c_void_p()
    _check(lib().scs_graph_create(C.byref(h), arr, len(items), prec))
    return h


def scs_graph_launch(graph, stream=None):
    if stream is None:
        stream = current_stream()
    _check(lib().scs_graph_launch(graph, _stream(stream)))


def scs_graph_destroy(graph):
    _check(lib().scs_graph_destroy(graph))


def scs_autotune_batch(items, prec=SCS_PREC_FP64, cache_path=None):
    """items: as scs_evaluate_batched."""
    arr = _items(items)
    _check(lib().scs_autotune_batch(arr, len(items), prec, cache_path.encode() if cache_path else None))


def scs_autotune(ctx, theta_cuda, N, prec=SCS_PREC_FP64, cache_path=None):
    need_f64(theta_cuda, "theta", (None, scs_ctx_info(ctx)["theta_dim"]))
    if not (_is_torch(theta_cuda) and theta_cuda.is_cuda and theta_cuda.is_contiguous()):
        raise ValueError("theta must be a contiguous CUDA tensor")
    _check(lib().scs_autotune(ctx, theta_cuda.shape[0], C.c_void_p(theta_cuda.data_ptr()), N, prec,
                              cache_path.encode() if cache_path else None))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check_box(ctx, lo, hi, periodic):
    D = scs_ctx_info(ctx)["theta_dim"]
    for name, x in (("lo", lo), ("hi", hi)) + ((("periodic", periodic),) if periodic is not None else ()):
        if np.asarray(x).shape != (D,):
            raise ValueError(f"{name} must have the context's {D} theta entries, got shape {np.asarray(x).shape}")


def scs_swarm_create(ctx, P, lo, hi, periodic=None, seed=0, swarm_id=0):
    _check_box(ctx, lo, hi, periodic)
    lo, hi = _f64(lo), _f64(hi)
    per = np.ascontiguousarray(periodic if periodic is not None else np.zeros(lo.size), dtype=np.int32)
    h = C.c_void_p()
    _check(lib().scs_swarm_create(ctx, C.byref(h), P, C.c_void_p(lo.ctypes.data), C.c_void_p(hi.ctypes.data),
                                  C.c_void_p(per.ctypes.data), seed, swarm_id))
    return h


def scs_swarm_destroy(sw):
    _check(lib().scs_swarm_destroy(sw))


def pso_params(omega, phi_p, phi_g, eps):
    """eps: 7 minimum speeds, or 8 (the last for e0) for eccentric swarms."""
    e = [float(x) for x in eps] + [0.0] * (8 - len(eps))
    return scs_pso_params(omega, phi_p, phi_g, (C.c_double * 8)(*e))


def scs_theta_dim(ctx):
    d = C.c_int32()
    _check(lib().scs_theta_dim(ctx, C.byref(d)))
    return d.value


def scs_search_create(ctx, n_swarms, particles, lo, hi, periodic=None, G=1, conv_tol=2.0, conv_window=50,
                      kmeans_iters=100, prec=SCS_PREC_FP64, seed=0):
    _check_box(ctx, lo, hi, periodic)
    prm = scs_search_params(n_swarms, G, particles, conv_tol, conv_window, kmeans_iters, prec, 0, seed)
    lo, hi = _f64(lo), _f64(hi)
    per = np.ascontiguousarray(periodic if periodic is not None else np.zeros(lo.size), dtype=np.int32)
    h = C.c_void_p()
    _check(lib().scs_search_create(ctx, C.byref(prm), C.c_void_p(lo.ctypes.data), C.c_void_p(hi.ctypes.data),
                                   C.c_void_p(per.ctypes.data), C.byref(h)))
    return h


def scs_search_run_rung(search, N, max_iters, params, stream=None):
    """One rung; returns the report as a dict."""
    r = scs_rung(N, max_iters, params)
    rep = scs_rung_report()
    _check(lib().scs_search_run_rung(search, C.byref(r), C.byref(rep), _stream(stream or current_stream())))
    return {k: getattr(rep, k) for k, _ in scs_rung_report._fields_}


def scs_search_swarms(search, max_swarms=64, dim=7):
    """(sizes [n], bests [n, dim + 1]: position, value); dim = the context's theta width."""
    n = C.c_int32()
    sizes = np.zeros(max_swarms, dtype=np.int64)
    best = np.zeros((max_swarms, dim + 1))
    _check(lib().scs_search_swarms(search, C.byref(n), C.c_void_p(sizes.ctypes.data), C.c_void_p(best.ctypes.data)))
    return sizes[:n.value].copy(), best[:n.value].copy()


def scs_search_destroy(search):
    _check(lib().scs_search_destroy(search))


def scs_kmeans(x, k, iters=100, seed=0):
    """x numpy [n, dim] -> (labels [n], centers [k_out, dim])."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n, dim = x.shape
    labels = np.empty(n, dtype=np.int32)
    centers = np.empty((k, dim))
    ko = C.c_int32()
    _check(lib().scs_kmeans(C.c_void_p(x.ctypes.data), n, dim, k, iters, seed, C.c_void_p(labels.ctypes.data),
                            C.c_void_p(centers.ctypes.data), C.byref(ko)))
    return labels, centers[:ko.value].copy()


def scs_kmeans_device(x, k, iters=100, seed=0, stream=None):
    """x torch float64 [n, dim] on the device -> (labels int32 [n], centers
    [k_out, dim]), both device tensors."""
    import torch

    if stream is None:
        stream = current_stream()
    if not (x.is_cuda and x.dtype == torch.float64 and x.dim() == 2 and x.is_contiguous()):
        raise ValueError("x must be a contiguous float64 [n, dim] device tensor")
    n, dim = x.shape
    labels = torch.empty(n, dtype=torch.int32, device=x.device)
    centers = torch.empty((k, dim), dtype=torch.float64, device=x.device)
    ko = C.c_int32()
    _check(lib().scs_kmeans_device(C.c_void_p(x.data_ptr()), n, dim, k, iters, seed, C.c_void_p(labels.data_ptr()),
                                   C.c_void_p(centers.data_ptr()), C.byref(ko), _stream(stream)))
    return labels, centers[:ko.value]


def scs_pso_step(sw, params, prec=SCS_PREC_FP64, stream=None):
    if stream is None:
        stream = current_stream()
    _check(lib().scs_pso_step(sw, C.byref(params), prec, _stream(stream)))


def scs_pso_step_swarms(sws, params, prec=SCS_PREC_FP64, stream=None, read_best=True):
    """One iteration of several swarms with one batched evaluation; returns
    each swarm's best value (numpy [n]) when read_best, else None."""
    if stream is None:
        stream = current_stream()
    arr = (C.c_void_p * len(sws))(*[sw.value if isinstance(sw, C.c_void_p) else sw for sw in sws])
    vals = np.empty(len(sws)) if read_best else None
    _check(lib().scs_pso_step_swarms(C.cast(arr, C.c_void_p), len(sws), C.byref(params), prec,
                                     C.c_void_p(vals.ctypes.data) if read_best else None, _stream(stream)))
    return vals


def scs_swarm_read(sw, P, dim=7):
    th, v, pb = np.empty((P, dim)), np.empty((P, dim)), np.empty((P, dim))
    pv, gb = np.empty(P), np.empty(dim)
    gv, it = C.c_double(), C.c_uint32()
    _check(lib().scs_swarm_read(sw, C.c_void_p(th.ctypes.data), C.c_void_p(v.ctypes.data),
                                C.c_void_p(pb.ctypes.data), C.c_void_p(pv.ctypes.data),
                                C.c_void_p(gb.ctypes.data), C.byref(gv), C.byref(it)))
    return {"theta": th, "vel": v, "pbest": pb, "pbest_val": pv, "gbest": gb, "gbest_val": gv.value,
            "iteration": it.value}


def scs_swarm_write(sw, state):
    arrs = [_f64(state[k]) for k in ("theta", "vel", "pbest", "pbest_val", "gbest")]
    _check(lib().scs_swarm_write(sw, *[C.c_void_p(a.ctypes.data) for a in arrs], float(state["gbest_val"]),
                                 int(state["iteration"])))


def scs_swarm_device_ptrs(sw):
    a, b = C.c_void_p(), C.c_void_p()
    _check(lib().scs_swarm_device_ptrs(sw, C.byref(a), C.byref(b)))
    return a.value, b.value


def _check_swarm_bufs(theta, **kw):
    need_f64(theta, "theta", (None, None))
    P, D = theta.shape
    if D not in (7, 8):
        raise ValueError("theta rows must have 7 or 8 entries")
    for name, (x, shape) in kw.items():
        need_f64(x, name, tuple(P if v == "P" else (D if v == "D" else v) for v in shape))
    for x in (theta, *(v[0] for v in kw.values())):
        if not (_is_torch(x) and x.is_cuda and x.is_contiguous()):
            raise ValueError("swarm buffers must be contiguous CUDA tensors")
    return P, D


def scs_pso_move(theta, vel, pbest, gbest, params, lo, hi, periodic, seed, swarm_id, iteration, stream=None):
    _check_swarm_bufs(theta, vel=(vel, ("P", "D")), pbest=(pbest, ("P", "D")), gbest=(gbest, ("D",)))
    lo, hi = _f64(lo), _f64(hi)
    per = np.ascontiguousarray(periodic, dtype=np.int32)
    if stream is None:
        stream = current_stream()
    _check(lib().scs_pso_move(theta.shape[0], theta.shape[1], theta.data_ptr(), vel.data_ptr(), pbest.data_ptr(),
                              gbest.data_ptr(),
                              C.byref(params), C.c_void_p(lo.ctypes.data), C.c_void_p(hi.ctypes.data),
                              C.c_void_p(per.ctypes.data), seed, swarm_id, iteration, _stream(stream)))


def scs_pso_best(theta, vals, lo, hi, periodic, pbest, pbest_val, gbest, gbest_val, stream=None):
    _check_swarm_bufs(theta, vals=(vals, ("P",)), pbest=(pbest, ("P", "D")), pbest_val=(pbest_val, ("P",)),
                      gbest=(gbest, ("D",)), gbest_val=(gbest_val, (1,)))
    lo, hi = _f64(lo), _f64(hi)
    per = np.ascontiguousarray(periodic, dtype=np.int32)
    if stream is None:
        stream = current_stream()
    _check(lib().scs_pso_best(theta.shape[0], theta.shape[1], theta.data_ptr(), vals.data_ptr(),
                              C.c_void_p(lo.ctypes.data),
                              C.c_void_p(hi.ctypes.data), C.c_void_p(per.ctypes.data), pbest.data_ptr(),
                              pbest_val.data_ptr(), gbest.data_ptr(), gbest_val.data_ptr(), _stream(stream)))


def scs_last_error():
    m = lib().scs_last_error()
    return m.decode() if m else ""


# ---------------------------------------------------------------- serving
def scs_server_create(device=0, max_inflight=16, hbm_budget=8 << 30, n_streams=4):
    h = C.c_void_p()
    _check(lib().scs_server_create(C.byref(h), device, max_inflight, hbm_budget, n_streams))
    return h


def scs_server_submit(srv, ctx, N, theta, ups, prec=SCS_PREC_FP64):
    """theta: numpy [P,7] float64 (copied); ups: numpy [P] float64, written when the request completes."""
    if not (isinstance(theta, np.ndarray) and isinstance(ups, np.ndarray)):
        raise TypeError("theta and ups must be numpy arrays (host memory)")
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    if theta.ndim != 2:
        raise ValueError("theta must be [P, D]")
    if ups.dtype != np.float64 or not ups.flags["C_CONTIGUOUS"] or ups.shape != (theta.shape[0],):
        raise ValueError("ups must be a contiguous float64 array of P entries")
    if ctx is not None:
        need_f64(theta, "theta", (None, scs_ctx_info(ctx)["theta_dim"]))
    rid = C.c_uint64()
    _check(lib().scs_server_submit(srv, ctx, N, theta.shape[0], C.c_void_p(theta.ctypes.data), prec,
                                   C.c_void_p(ups.ctypes.data), C.byref(rid)))
    return rid.value


def scs_server_poll(srv, max_out=256, wait_ms=0):
    """List of dicts (id, status, t_submit, t_admit, t_launch, t_done) of finished requests."""
    arr = (scs_request_done * max_out)()
    n = C.c_int32()
    _check(lib().scs_server_poll(srv, arr, max_out, wait_ms, C.byref(n)))
    return [{k: getattr(arr[i], k) for k in ("id", "status", "t_submit", "t_admit", "t_launch", "t_done")}
            for i in range(n.value)]


def scs_server_stats(srv):
    c = scs_server_counters()
    _check(lib().scs_server_stats(srv, C.byref(c)))
    return {k: getattr(c, k) for k, _ in scs_server_counters._fields_}


def scs_server_clock(srv):
    return lib().scs_server_clock(srv)


def scs_server_destroy(srv):
    _check(lib().scs_server_destroy(srv))


def scs_peak_probe(device=0):
    """Measured device ceilings: FP64 and FP32 FMA TFLOP/s, FP32 sines per
    second (1e12), HBM copy TB/s (read + write), HIP's clock in GHz."""
    out = np.zeros(5)
    _check(lib().scs_peak_probe(device, out.ctypes.data_as(C.POINTER(C.c_double))))
    return {"fp64_tflops": out[0], "fp32_tflops": out[1], "sin32_per_s_1e12": out[2], "hbm_copy_tbps": out[3],
            "clock_ghz": out[4]}
