"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the statistic itself: it only describes
the workloads (grids, priors, injected parameters) and draws random numbers
(Gaussian frequency-domain noise coloured by a PSD, particles uniform in a
prior box).  The injected signal is added by the caller, which generates the
template with whichever implementation it is allowed to use.

Workload recipe (stands in for the paper's mock LISA data, Sec 4):
  * grid: K uniform bins from f_min = 0.016 Hz, df = (0.032 - 0.016) / K,
    T_obs = 1 / df;
  * noise: stationary Gaussian, generated directly in the frequency domain
    from a known PSD (Sec 4, noise paragraph), n = sqrt(S / (4 df)) (a + i b)
    with a, b standard normal, so that <n|h> ~ N(0, <h|h>);
  * PSD: unit white (single channel) or the two-component LISA instrument
    model (OMS 15 pm/rtHz, acceleration 3 fm/s^2/rtHz, L = 2.5e9 m) for the
    A and E channels, S_A = S_E = 1.5 P_n(f);
  * particles: uniform in the prior box of Table tab:GW150914-like_injection
    (or the small chirp-mass / mass-ratio box of the single-channel case).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 2408131

THETA_NAMES = ("Mc", "eta", "f_low", "lambda", "beta", "iota", "psi")

# Table tab:GW150914-like_injection (circular: e0 dropped)
GW150914_LIKE = np.array([28.095555, 0.2471, 0.018, 2.01, math.pi / 4, 2.498, -1.85])
GW150914_PRIOR_LO = np.array([27.0, 0.15, 0.0178, 0.0, -math.pi / 2, 0.0, -math.pi])
GW150914_PRIOR_HI = np.array([30.0, 0.2495, 0.0182, 2 * math.pi, math.pi / 2, math.pi, 0.0])
# Table tab:GW190521-like_injection
GW190521_LIKE = np.array([95.0209, 0.234, 0.0175, 3.24, 0.4, 2.0, -1.5])
GW190521_PRIOR_LO = np.array([93.0, 0.15, 0.014, 0.0, -math.pi / 2, 0.0, -math.pi])
GW190521_PRIOR_HI = np.array([96.0, 0.2495, 0.019, 2 * math.pi, math.pi / 2, math.pi, 0.0])
# periodic dimensions of the swarm: lambda (2 pi) and psi (pi)
PERIODIC = np.array([0, 0, 0, 1, 0, 0, 1], dtype=np.int32)

F_MIN = 0.016
F_MAX = 0.032


def eta_from_q(q):
    """Symmetric mass ratio from q = m2/m1 <= 1."""
    q = np.asarray(q, dtype=np.float64)
    return q / (1.0 + q) ** 2


def lisa_pn(f, L=2.5e9, s_oms=15e-12, s_acc=3e-15):
    """Single-link-pair (Michelson) two-component instrument noise P_n(f)
    [1/Hz] (Robson, Cornish & Liu 2019 form without the transfer function)."""
    f = np.asarray(f, dtype=np.float64)
    c = 299792458.0
    fstar = c / (2 * math.pi * L)
    p_oms = s_oms ** 2 * (1.0 + (2e-3 / f) ** 4)
    p_acc = s_acc ** 2 * (1.0 + (0.4e-3 / f) ** 2) * (1.0 + (f / 8e-3) ** 4)
    return p_oms / L ** 2 + 2.0 * (1.0 + np.cos(f / fstar) ** 2) * p_acc / ((2 * math.pi * f) ** 4 * L ** 2)


def lisa_tdi_psd(f, L=2.5e9, s_oms=15e-12, s_acc=3e-15):
    """Noise PSDs [3, len(f)] of the A, E and T channels of first-generation
    TDI on an equal-arm constellation (uncorrelated optical-metrology noise on
    each of the six links, acceleration noise on each of the six test masses,
    the same two-component levels as ``lisa_pn``), in fractional frequency
    S_A = S_E = 8 sin^2 x [(2 + cos x) S_oms + 2 (3 + 2 cos x + cos 2x) S_acc],
    S_T = 32 sin^2 x sin^2(x/2) [S_oms + 4 sin^2(x/2) S_acc], x = 2 pi f L / c,
    then divided by 16 x^4: the normalisation of the full response's
    channels (TDI / (4 x^2)), under which A and E tend to 1.5 P_n at low f."""
    f = np.asarray(f, dtype=np.float64)
    c = 299792458.0
    x = 2 * math.pi * f * L / c
    oms = s_oms ** 2 * (2 * math.pi * f / c) ** 2 * (1.0 + (2e-3 / f) ** 4)
    acc = s_acc ** 2 / (2 * math.pi * f * c) ** 2 * (1.0 + (0.4e-3 / f) ** 2) * (1.0 + (f / 8e-3) ** 4)
    sa = 8 * np.sin(x) ** 2 * ((2 + np.cos(x)) * oms + 2 * (3 + 2 * np.cos(x) + np.cos(2 * x)) * acc)
    st = 32 * np.sin(x) ** 2 * np.sin(x / 2) ** 2 * (oms + 4 * np.sin(x / 2) ** 2 * acc)
    return np.stack([sa, sa, st]) / (16 * x ** 4)


@dataclass
class GridSpec:
    K: int
    f_min: float = F_MIN
    f_max: float = F_MAX

    @property
    def df(self):
        return (self.f_max - self.f_min) / self.K

    @property
    def k0(self):
        return int(round(self.f_min / self.df))

    @property
    def t_obs(self):
        return 1.0 / self.df

    def freqs(self):
        return (self.k0 + np.arange(self.K, dtype=np.float64)) * self.df


@dataclass
class Workload:
    name: str
    grid: GridSpec
    n_chan: int
    pn_order: int
    response: int  # 0 none, 1 LISA low-frequency A/E
    support: int  # 0 full band, 1 observation window
    N: int
    P: int
    G: int
    snr: float
    injection: np.ndarray
    prior_lo: np.ndarray
    prior_hi: np.ndarray
    seed: int
    white: bool = False
    extra: dict = field(default_factory=dict)


def single_channel_box():
    """Single-channel case: Mc in 30 [0.99, 1.01], q in 0.8 [0.9, 1.1];
    f_low = f_min; sky and polarisation unused."""
    lo = np.array([30 * 0.99, float(eta_from_q(0.72)), F_MIN, 0.0, 0.0, 0.0, 0.0])
    hi = np.array([30 * 1.01, float(eta_from_q(0.88)), F_MIN, 0.0, 0.0, 0.0, 0.0])
    return lo, hi


def workload(name: str) -> Workload:
    """The workloads.  'white16k': single channel, 16384 bins, unit white PSD,
    2PN, whole-band support, N = 16, 64 particles.  'lisa1m': A+E, 2^20 bins,
    two-component PSD, 3.5PN, low-frequency response, observation-window
    support, N = 1024, 10^4 particles from the GW150914-like prior box."""
    if name == "white16k":
        lo, hi = single_channel_box()
        inj = np.array([30.0, float(eta_from_q(0.8)), F_MIN, 0.0, 0.0, 0.0, 0.0])
        return Workload(name, GridSpec(16384), 1, 4, 0, 0, 16, 64, 1, 20.0, inj, lo, hi,
                        BASE_SEED + 1, white=True)
    if name == "lisa1m":
        return Workload(name, GridSpec(1 << 20), 2, 7, 1, 1, 1024, 10000, 1024, 17.0,
                        GW150914_LIKE.copy(), GW150914_PRIOR_LO.copy(), GW150914_PRIOR_HI.copy(),
                        BASE_SEED + 2)
    raise KeyError(name)


# Batched hierarchy: six swarms (N, P)
LADDER_SWARMS = [(4096, 16384), (1024, 8192), (256, 4096), (64, 2048), (16, 512), (1, 128)]


def psd_arrays(w: Workload):
    f = w.grid.freqs()
    if w.white:
        return np.ones((w.n_chan, w.grid.K))
    s = 1.5 * lisa_pn(f)
    return np.stack([s] * w.n_chan)


def noise(psd, df, seed):
    """Frequency-domain Gaussian noise [n_chan, K] complex, <n|h> ~ N(0, <h|h>)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(psd.shape)
    b = rng.standard_normal(psd.shape)
    return np.sqrt(psd / (4.0 * df)) * (a + 1j * b)


def particles(lo, hi, P, seed):
    """P points uniform in the box [lo, hi] (dimensions with lo == hi are fixed)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    u = rng.random((P, lo.size))
    return lo + u * (hi - lo)


def single_channel_particles(P, seed):
    """Mc uniform in 30 [0.99, 1.01], q uniform in 0.8 [0.9, 1.1] -> eta."""
    rng = np.random.default_rng(seed)
    mc = 30.0 * (0.99 + 0.02 * rng.random(P))
    q = 0.8 * (0.9 + 0.2 * rng.random(P))
    th = np.zeros((P, 7))
    th[:, 0] = mc
    th[:, 1] = eta_from_q(np.minimum(q, 1.0))
    th[:, 2] = F_MIN
    return th


def near_injection(inj, P, seed, rel=1e-4, lo=None, hi=None):
    """Particles jittered around an injection (peak-accuracy checks)."""
    rng = np.random.default_rng(seed)
    th = np.tile(np.asarray(inj, dtype=np.float64), (P, 1))
    scale = np.array([1e-3, 1e-3, 1e-6, 1e-2, 1e-2, 1e-2, 1e-2]) * rel / 1e-4
    th = th + rng.standard_normal(th.shape) * scale
    if lo is not None:
        th = np.clip(th, lo, hi)
    th[:, 1] = np.minimum(th[:, 1], 0.25)
    return th


def workload_particles(w: Workload, P=None, seed=None):
    P = w.P if P is None else P
    seed = w.seed + 100 if seed is None else seed
    if w.name == "white16k":
        return single_channel_particles(P, seed)
    return particles(w.prior_lo, w.prior_hi, P, seed)


def served_streams():
    """Eight independent served searches: K cycles over 2^19, 2^20, 2^21,
    alternating GW150914-like / GW190521-like injections with seeded jitter,
    SNR from 15 to 40."""
    snrs = [15, 17, 20, 22, 25, 30, 35, 40]
    out = []
    for i in range(8):
        K = 1 << (19 + (i % 3))
        rng = np.random.default_rng(BASE_SEED + 500 + i)
        if i % 2 == 0:
            inj, lo, hi = GW150914_LIKE.copy(), GW150914_PRIOR_LO, GW150914_PRIOR_HI
        else:
            inj, lo, hi = GW190521_LIKE.copy(), GW190521_PRIOR_LO, GW190521_PRIOR_HI
        inj = inj + (hi - lo) * 0.01 * (rng.random(7) - 0.5)
        inj[1] = min(inj[1], 0.2495)
        w = Workload(f"served{i}", GridSpec(K), 2, 7, 1, 1, 1024, 0, 1024, float(snrs[i]), inj,
                     lo.copy(), hi.copy(), BASE_SEED + 600 + i)
        out.append(w)
    return out
