"""Plain CPU oracle for the semi-coherent statistic Upsilon_N (arXiv:2408.13170).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library ``paper_2408_13170_amd`` and neither imports the
other.  The arithmetic lives in ``oracle.c`` (built by ``oracle/build.py``);
this module only marshals numpy arrays through ctypes.

Besides Upsilon_N it gives the likelihood quantities of Sec 2.1 - 2.2
(``data_norm``, ``likelihood_stats``, ``loglike``), written in numpy on top of
the per-segment sums of ``evaluate``.  ``oracle/search.py`` is the
hierarchical multi-swarm search of Sec 3.2 over a caller-given objective.

Parameter vector theta (7 doubles):
    Mc [Msun, detector frame], eta, f_low [Hz], lambda, beta, iota, psi
(the searched parameters of Table tab:GW150914-like_injection, without e0).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liborc.so")
_lib = None

SEG_EQUAL_SNR = 0
SEG_UNIFORM = 1
SEG_EXPLICIT = 2

RESP_NONE = 0
RESP_LISA_LF_AE = 1
RESP_LISA_FD = 2

SUPPORT_FULL = 0
SUPPORT_TOBS = 1


class _Grid(C.Structure):
    _fields_ = [("K", C.c_int64), ("k0", C.c_int64), ("df", C.c_double),
                ("n_chan", C.c_int32), ("pad", C.c_int32)]


class _Model(C.Structure):
    _fields_ = [("pn_order", C.c_int32), ("response", C.c_int32), ("support", C.c_int32),
                ("eccentric", C.c_int32), ("t_obs", C.c_double), ("orbit_phase0", C.c_double),
                ("cartwheel_phase0", C.c_double), ("sparse_stride", C.c_int32), ("pad", C.c_int32)]


@dataclass
class Grid:
    K: int
    k0: int
    df: float
    n_chan: int

    def c(self):
        return _Grid(self.K, self.k0, self.df, self.n_chan, 0)

    @property
    def freqs(self):
        return (self.k0 + np.arange(self.K, dtype=np.float64)) * self.df


@dataclass
class Model:
    pn_order: int = 7
    response: int = RESP_LISA_LF_AE
    support: int = SUPPORT_TOBS
    t_obs: float = 0.0
    orbit_phase0: float = 0.0
    cartwheel_phase0: float = 0.0
    eccentric: int = 0  # 1: theta rows carry an 8th entry, e0 at GW frequency f_low
    # 0: template evaluated at every bin; S > 0: the sparse-grid evaluation of
    # Sec 4 (phase and response at every S-th bin of the support and its ends,
    # not-a-knot cubic splines onto every bin)
    sparse_stride: int = 0

    @property
    def theta_dim(self):
        return 8 if self.eccentric else 7

    def c(self):
        return _Model(self.pn_order, self.response, self.support, int(self.eccentric), self.t_obs,
                      self.orbit_phase0, self.cartwheel_phase0, int(self.sparse_stride), 0)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIBPATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int64)
        L.orc_evaluate.argtypes = [C.POINTER(_Grid), C.POINTER(_Model), dp, dp, C.c_int64, dp,
                                   C.c_int32, C.c_int32, C.c_int32, ip, dp, dp, ip, ip, C.c_int32]
        L.orc_evaluate.restype = C.c_int
        L.orc_edge_cumulative.argtypes = [C.POINTER(_Grid), C.POINTER(_Model), dp, dp, C.c_int32, C.c_int64, ip,
                                          dp, dp, ip]
        L.orc_edge_cumulative.restype = C.c_int
        L.orc_template.argtypes = [C.POINTER(_Grid), C.POINTER(_Model), dp, dp]
        L.orc_template.restype = C.c_int
        L.orc_phase.argtypes = [C.POINTER(_Model), dp, C.c_int64, dp, dp, dp, dp, dp]
        L.orc_phase.restype = C.c_int
        L.orc_phase_bins.argtypes = [C.POINTER(_Grid), C.POINTER(_Model), dp, C.c_int64, ip, dp, dp]
        L.orc_phase_bins.restype = C.c_int
        L.orc_response.argtypes = [C.POINTER(_Model), dp, C.c_double, dp, dp, dp]
        L.orc_response.restype = C.c_int
        L.orc_fd_transfer.argtypes = [C.POINTER(_Model), dp, C.c_double, C.c_double, dp]
        L.orc_fd_transfer.restype = C.c_int
        u32p = C.POINTER(C.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_uniform.restype = C.c_double
        i32p = C.POINTER(C.c_int32)
        L.orc_pso_init.argtypes = [C.c_int64, C.c_int32, dp, dp, C.c_uint64, C.c_uint32, dp]
        L.orc_pso_init.restype = None
        L.orc_pso_move.argtypes = [C.c_int64, C.c_int32, dp, dp, dp, dp, C.c_double, C.c_double,
                                   C.c_double, dp, dp, dp, i32p, C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_pso_move.restype = None
        L.orc_pso_best.argtypes = [C.c_int64, C.c_int32, dp, dp, dp, dp, i32p, dp, dp, dp, dp]
        L.orc_pso_best.restype = None
        L.orc_noise.argtypes = [C.c_int64, C.c_int32, dp, C.c_double, C.c_uint64, C.c_uint32, dp]
        L.orc_noise.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def evaluate(grid: Grid, model: Model, d_ri, psd, theta, N, mode=SEG_EQUAL_SNR, G=1,
             edges=None, want_seg=False, want_bounds=False, n_threads=0):
    """Upsilon_N for every row of theta [P,7].  Returns dict with 'ups' and,
    on request, 'seg' [P,N,3] = (Re Z_n, Im Z_n, H_n), 'bounds' [P,N+1],
    'support' [P,2]."""
    d_ri = _f64(d_ri)
    psd = _f64(psd)
    theta = _f64(theta).reshape(-1, model.theta_dim)
    P = theta.shape[0]
    assert d_ri.shape == (grid.n_chan, grid.K, 2)
    assert psd.shape == (grid.n_chan, grid.K)
    ups = np.empty(P)
    seg = np.empty((P, N, 3)) if want_seg else None
    bnd = np.empty((P, N + 1), dtype=np.int64) if want_bounds else None
    sup = np.empty((P, 2), dtype=np.int64)
    e = None
    if mode == SEG_EXPLICIT:
        e = np.ascontiguousarray(edges, dtype=np.int64)
        assert e.shape == (N + 1,)
    g, m = grid.c(), model.c()
    rc = lib().orc_evaluate(C.byref(g), C.byref(m), _dp(d_ri), _dp(psd), P, _dp(theta), N, mode,
                            G, _ip(e), _dp(ups), _dp(seg), _ip(bnd), _ip(sup), n_threads)
    if rc != 0:
        raise ValueError(f"orc_evaluate failed ({rc})")
    out = {"ups": ups, "support": sup}
    if want_seg:
        out["seg"] = seg
    if want_bounds:
        out["bounds"] = bnd
    return out


def edge_cumulative(grid: Grid, model: Model, psd, theta, G, ks):
    """The equal-[h|h] edge rule's cumulative C(k) of one particle at bins ks
    (clamped to its support), its total C(k_hi) and the support (k_lo, k_hi).
    The rule: nodes k_lo + jG and k_hi - 1, weights linear between nodes,
    C(k) = sum of the weights of bins k_lo..k-1 (Sec 2.2, equal [h|h] per
    segment)."""
    psd = _f64(psd)
    theta = _f64(theta).reshape(model.theta_dim)
    k = np.ascontiguousarray(np.atleast_1d(ks), dtype=np.int64)
    Ck = np.empty(k.size)
    tot = C.c_double()
    sup = np.empty(2, dtype=np.int64)
    g, m = grid.c(), model.c()
    rc = lib().orc_edge_cumulative(C.byref(g), C.byref(m), _dp(psd), _dp(theta), int(G), k.size, _ip(k),
                                   _dp(Ck), C.byref(tot), _ip(sup))
    if rc != 0:
        raise ValueError(f"orc_edge_cumulative failed ({rc})")
    return Ck, tot.value, (int(sup[0]), int(sup[1]))


def data_norm(grid: Grid, d_ri, psd):
    """<d|d> = sum_alpha 4 df sum_k |d_alpha(f_k)|^2 / S_alpha(f_k)
    (eqn:inner_prod with a = b = d, rectangle rule on the bins)."""
    d_ri, psd = _f64(d_ri), _f64(psd)
    return float(4.0 * grid.df * np.sum((d_ri[..., 0] ** 2 + d_ri[..., 1] ** 2) / psd))


def likelihood_stats(grid: Grid, model: Model, d_ri, psd, theta, N, mode=SEG_EQUAL_SNR, G=1, edges=None):
    """Sufficient statistics of the likelihoods of Sec 2.1 - 2.2 for every row
    of theta, for the template h of ``template()`` at unit amplitude and zero
    phase offset; with Z_n = sum over segment n of d conj(h) / S and
    H_n = sum |h|^2 / S (the per-segment sums of ``evaluate``):
        ups      Upsilon_N = sum_n x_n^2 / [h|h]_n
        overlap  hat O_N(d, h) = sum_n max_phi_n [d|h e^{i phi_n}]_n
                 = sum_n 4 df |Z_n|                       (eq:semi-coherent_O)
        hh       <h|h> = sum_n [h|h]_n = 4 df sum_n H_n    (eqn:SNR_coherent, squared)
        dh       <d|h> as a complex number 4 df sum_n Z_n, so that
                 <d|h e^{i phi}> = Re(e^{-i phi} dh)       (eqn:inner_prod)
    Returns a dict of [P] arrays (dh complex; 'bounds' [P, N+1] the edges);
    NaN rows for invalid theta."""
    out = evaluate(grid, model, d_ri, psd, theta, N, mode, G, edges, want_seg=True, want_bounds=True)
    seg = out["seg"]
    Z = seg[..., 0] + 1j * seg[..., 1]
    H = seg[..., 2]
    w = 4.0 * grid.df
    return {"ups": out["ups"], "overlap": w * np.sum(np.abs(Z), axis=1), "hh": w * np.sum(H, axis=1),
            "dh": w * np.sum(Z, axis=1), "bounds": out["bounds"]}


# IAU nominal solar mass parameter, speed of light, parsec (648000/pi au)
_GM_SUN = 1.32712440018e20   # m^3 s^-2
_C = 299792458.0             # m s^-1
_MPC = 3.0856775814913673e22  # m


def distance_amplitude(mc_msun, dl_mpc):
    """Absolute amplitude of the template h = f^-7/6 R e^{-i Psi} (the
    response R carrying (1 + cos^2 iota)/2 and cos iota) for a source at
    luminosity distance D_L: the restricted stationary-phase amplitude of the
    (2,2) mode, sqrt(5/24) pi^-2/3 (G Mc / c^3)^5/6 c / D_L, with Mc the
    detector-frame chirp mass (Sec 4: D_L is a 1/D_L prefactor of the
    amplitude; Sec 2.1, eqn:LogL_coherent needs the absolute amplitude)."""
    mc = np.asarray(mc_msun, dtype=np.float64)
    dl = np.asarray(dl_mpc, dtype=np.float64)
    ok = (mc > 0) & (dl > 0) & np.isfinite(mc) & np.isfinite(dl)
    tm = np.where(ok, mc, 1.0) * _GM_SUN / _C ** 3  # s
    a = np.sqrt(5.0 / 24.0) * np.pi ** (-2.0 / 3.0) * tm ** (5.0 / 6.0) * _C / (np.where(ok, dl, 1.0) * _MPC)
    return np.where(ok, a, np.nan)  # no physical amplitude for Mc <= 0 or D_L <= 0


def loglike(dd, stats, amp, phase=None):
    """Log-likelihoods for templates A h e^{i phi} (A real), dropping the
    normalisation constant as the paper does:
        semi  log hat L_N = -<d|d>/2 - A^2 <h|h>/2 + hat O_N(d, A h)
                          = -<d|d>/2 - A^2 <h|h>/2 + |A| hat O_N(d, h)
        coh   log L       = -<d|d>/2 - A^2 <h|h>/2 + A Re(e^{-i phi} <d|h>)   (eqn:LogL_coherent)
    With phase None the coherent one is maximised over phi (|A| |<d|h>|)."""
    amp = np.asarray(amp, dtype=np.float64)
    base = -0.5 * dd - 0.5 * amp ** 2 * stats["hh"]
    semi = base + np.abs(amp) * stats["overlap"]
    if phase is None:
        coh = base + np.abs(amp) * np.abs(stats["dh"])
    else:
        coh = base + amp * np.real(np.exp(-1j * np.asarray(phase, dtype=np.float64)) * stats["dh"])
    return semi, coh


def noise(grid: Grid, psd, seed, r):
    """Noise realisation r [n_chan, K] complex: sqrt(S / (4 df)) (g1 + i g2) with
    Box-Muller normals from Philox4x32-10, counter (k, channel, r, stream), key seed
    (the generator the GPU's realisation kernel implements on its own)."""
    psd = _f64(psd)
    out = np.empty((grid.n_chan, grid.K, 2))
    lib().orc_noise(grid.K, grid.n_chan, _dp(psd), grid.df, seed, r, _dp(out))
    return out[..., 0] + 1j * out[..., 1]


def template(grid: Grid, model: Model, theta):
    """h_alpha(f_k) over the grid, complex array [n_chan, K] (zero off support)."""
    theta = _f64(theta).reshape(model.theta_dim)
    h = np.zeros((grid.n_chan, grid.K, 2))
    g, m = grid.c(), model.c()
    rc = lib().orc_template(C.byref(g), C.byref(m), _dp(theta), _dp(h))
    if rc != 0:
        raise ValueError("invalid theta")
    return h[..., 0] + 1j * h[..., 1]


def phase(model: Model, theta, f_hz):
    """(phase mod 1 [cycles], integer part, SPA time [s], t_c [s]) at frequencies f_hz."""
    theta = _f64(theta).reshape(model.theta_dim)
    f = _f64(np.atleast_1d(f_hz))
    fr, it, t = np.empty_like(f), np.empty_like(f), np.empty_like(f)
    tc = C.c_double()
    m = model.c()
    rc = lib().orc_phase(C.byref(m), _dp(theta), f.size, _dp(f), _dp(fr), _dp(it), _dp(t), C.byref(tc))
    if rc != 0:
        raise ValueError("invalid theta")
    return fr, it, t, tc.value


def phase_bins(grid: Grid, model: Model, theta, bins):
    theta = _f64(theta).reshape(model.theta_dim)
    b = np.ascontiguousarray(bins, dtype=np.int64)
    fr, t = np.empty(b.size), np.empty(b.size)
    g, m = grid.c(), model.c()
    rc = lib().orc_phase_bins(C.byref(g), C.byref(m), _dp(theta), b.size, _ip(b), _dp(fr), _dp(t))
    if rc != 0:
        raise ValueError("invalid theta")
    return fr, t


def response(model: Model, theta, t):
    """(F [2 chan, 2 pol], Doppler cycles per Hz, T-channel (F+, Fx)) at time t."""
    theta = _f64(theta).reshape(model.theta_dim)
    F = np.empty(4)
    dop = C.c_double()
    tch = np.empty(2)
    m = model.c()
    rc = lib().orc_response(C.byref(m), _dp(theta), float(t), _dp(F), C.byref(dop), _dp(tch))
    if rc != 0:
        raise ValueError("invalid theta")
    return F.reshape(2, 2), dop.value, tch


def fd_transfer(model: Model, theta, f, t):
    """Full-response transfer functions (A, E, T), complex [3], at frequency
    f [Hz] and time t [s] (response 2)."""
    theta = _f64(theta).reshape(model.theta_dim)
    R = np.empty(6)
    m = model.c()
    if lib().orc_fd_transfer(C.byref(m), _dp(theta), float(f), float(t), _dp(R)) != 0:
        raise ValueError("invalid theta")
    return R[0::2] + 1j * R[1::2]


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def uniform(seed, swarm, it, particle, dim, stream):
    return lib().orc_uniform(seed, swarm, it, particle, dim, stream)


def pso_init(P, lo, hi, seed, swarm):
    lo, hi = _f64(lo), _f64(hi)
    D = lo.size
    th = np.empty((P, D))
    lib().orc_pso_init(P, D, _dp(lo), _dp(hi), seed, swarm, _dp(th))
    return th


def pso_move(theta, vel, pbest, gbest, omega, phi_p, phi_g, eps, lo, hi, periodic, seed, swarm, it):
    """In-place synchronous PSO move (eqn:PSO_velocity_rule, eqn:PSO_min_velocity)."""
    P, D = theta.shape
    per = np.ascontiguousarray(periodic, dtype=np.int32)
    lib().orc_pso_move(P, D, _dp(theta), _dp(vel), _dp(_f64(pbest)), _dp(_f64(gbest)), omega, phi_p,
                       phi_g, _dp(_f64(eps)), _dp(_f64(lo)), _dp(_f64(hi)),
                       per.ctypes.data_as(C.POINTER(C.c_int32)), seed, swarm, it)


def pso_best(theta, vals, lo, hi, periodic, pbest, pbest_val, gbest, gbest_val):
    """In-place best update; returns the new swarm-best value."""
    P, D = theta.shape
    per = np.ascontiguousarray(periodic, dtype=np.int32)
    gv = np.array([gbest_val], dtype=np.float64)
    lib().orc_pso_best(P, D, _dp(_f64(theta)), _dp(_f64(vals)), _dp(_f64(lo)), _dp(_f64(hi)),
                       per.ctypes.data_as(C.POINTER(C.c_int32)), _dp(pbest), _dp(pbest_val),
                       _dp(gbest), _dp(gv))
    return float(gv[0])
