"""Seeded test datasets: noise from ``synth``, injections from the oracle.

Inputs and expected values here never come from the HIP library.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle as O
import synth


@dataclass
class Dataset:
    grid: O.Grid
    model: O.Model
    psd: np.ndarray  # [n_chan, K]
    d: np.ndarray  # complex [n_chan, K]
    injection: np.ndarray
    snr: float
    lo: np.ndarray
    hi: np.ndarray

    @property
    def d_ri(self):
        return np.stack([self.d.real, self.d.imag], axis=-1)

    @property
    def f_min(self):
        return self.grid.k0 * self.grid.df


def inner(grid, psd, a, b):
    """<a|b> = 4 df Re sum a conj(b) / S  (eqn:inner_prod, rectangle rule)."""
    return 4.0 * grid.df * float(np.real(np.sum(a * np.conj(b) / psd)))


def make(grid: O.Grid, model: O.Model, psd, injection, snr, seed, noise=True, lo=None, hi=None):
    """Data = noise (seeded) + injection scaled to optimal SNR `snr`."""
    h = O.template(grid, model, injection)
    hh = inner(grid, psd, h, h)
    d = np.zeros((grid.n_chan, grid.K), dtype=np.complex128)
    if snr > 0 and hh > 0:
        d += h * (snr / np.sqrt(hh))
    if noise:
        d += synth.noise(psd, grid.df, seed)
    return Dataset(grid, model, psd, d, np.asarray(injection, float), snr, lo, hi)


def white_small(K=1024, pn_order=4, snr=20.0, seed=11, noise=True):
    """Single channel, unit white PSD, whole-band support (the 16384-bin
    workload shrunk to K bins)."""
    spec = synth.GridSpec(K)
    grid = O.Grid(K, spec.k0, spec.df, 1)
    model = O.Model(pn_order=pn_order, response=O.RESP_NONE, support=O.SUPPORT_FULL, t_obs=spec.t_obs)
    lo, hi = synth.single_channel_box()
    inj = np.array([30.0, float(synth.eta_from_q(0.8)), spec.f_min, 0, 0, 0, 0])
    return make(grid, model, np.ones((1, K)), inj, snr, seed, noise, lo, hi)


def white16k(seed=None, noise=True):
    w = synth.workload("white16k")
    grid = O.Grid(w.grid.K, w.grid.k0, w.grid.df, 1)
    model = O.Model(pn_order=w.pn_order, response=O.RESP_NONE, support=O.SUPPORT_FULL, t_obs=w.grid.t_obs)
    return make(grid, model, synth.psd_arrays(w), w.injection, w.snr,
                w.seed if seed is None else seed, noise, w.prior_lo, w.prior_hi)


def lisa_small(K=20000, df=1e-7, f_min=0.017, pn_order=7, snr=17.0, seed=21, noise=True, t_obs=None,
               response=O.RESP_LISA_LF_AE, n_chan=2):
    """A+E low-frequency response on a short band around the GW150914-like
    source: f in [0.017, 0.019) Hz at df = 1e-7 Hz (T_obs = 1e7 s), so that the
    observation window covers a few thousand bins.  With the full response,
    A+E (n_chan 2) or A+E+T (n_chan 3) and the TDI noise PSDs."""
    k0 = int(round(f_min / df))
    grid = O.Grid(K, k0, df, n_chan)
    model = O.Model(pn_order=pn_order, response=response, support=O.SUPPORT_TOBS,
                    t_obs=(1.0 / df) if t_obs is None else t_obs)
    f = (k0 + np.arange(K)) * df
    if response == O.RESP_LISA_FD:
        psd = synth.lisa_tdi_psd(f)[:n_chan]
    else:
        s = 1.5 * synth.lisa_pn(f)
        psd = np.stack([s, s])
    return make(grid, model, psd, synth.GW150914_LIKE, snr, seed, noise,
                synth.GW150914_PRIOR_LO, synth.GW150914_PRIOR_HI)


def lisa_particles(n, seed, near=None):
    """Particles from the GW150914-like prior box, with the lower-frequency
    edge restricted so that the short test band still holds their support."""
    lo = synth.GW150914_PRIOR_LO.copy()
    hi = synth.GW150914_PRIOR_HI.copy()
    th = synth.particles(lo, hi, n, seed)
    if near is not None:
        th[: near.shape[0]] = near
    return th
