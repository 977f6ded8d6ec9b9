"""Pins of the oracle's eccentric phase (the TaylorF2Ecc model named in Sec 4,
kept at its leading order in e0^2 and Newtonian order).

The correction is fixed from outside the oracle by the Peters-Mathews
evolution of orbital frequency F and eccentricity e (Peters 1964):
    dF/dt = (48 / (5 pi)) Mc^(5/3) (2 pi F)^(11/3) (1 + 73/24 e^2 + 37/96 e^4) / (1 - e^2)^(7/2),
    de/dt = -(1/15) Mc^(5/3) (2 pi F)^(8/3) e (304 + 121 e^2) / (1 - e^2)^(5/2)
(Mc in seconds), integrated numerically; the GW frequency of the dominant
harmonic is f = 2F.  The stationary-phase time t(f) of the oracle must follow
the integrated t(F) up to O(e0^4), and so must its phase: in the stationary-
phase approximation Psi(f)/2pi = f t(f) - Phi(f) + const, where Phi(f) is the
number of GW cycles emitted up to the time the frequency is f, which the same
evolution gives as the integral of f dt.  The phase and the time are written
as separate terms in the oracle, so the two are pinned one by one, and their
consistency (t = Psi'/2pi) is checked on the eccentric model as well.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests import datasets as D

scipy_integrate = pytest.importorskip("scipy.integrate")

TSUN = 1.32712440018e20 / 299792458.0 ** 3


def _model(ecc, pn=0, response=O.RESP_NONE):
    return O.Model(pn_order=pn, response=response, support=O.SUPPORT_FULL, t_obs=1e8, eccentric=ecc)


def _theta(mc, flow, e0):
    return np.array([mc, 0.24, flow, 0.0, 0.0, 0.0, 0.0, e0])


def _peters_mathews(mc, f0, e0, freqs):
    """t(f) - t(f0) and the GW cycles Phi(f) - Phi(f0) from the
    Peters-Mathews equations, integrated in the orbital frequency F
    (dt/dF = 1/Fdot, dPhi/dF = 2F/Fdot: the dominant harmonic has twice the
    orbital frequency)."""
    mcs = mc * TSUN

    def rhs(F, y):
        t, e, _ = y
        w = 2 * math.pi * F
        fdot = 48 / (5 * math.pi) * mcs ** (5 / 3) * w ** (11 / 3) * (1 + 73 / 24 * e * e + 37 / 96 * e ** 4) / (
            1 - e * e) ** 3.5
        edot = -mcs ** (5 / 3) * w ** (8 / 3) * e * (304 + 121 * e * e) / (15 * (1 - e * e) ** 2.5)
        return [1.0 / fdot, edot / fdot, 2.0 * F / fdot]

    sol = scipy_integrate.solve_ivp(rhs, (f0 / 2, freqs[-1] / 2), [0.0, e0, 0.0], t_eval=np.asarray(freqs) / 2,
                                    rtol=1e-13, atol=1e-14, method="DOP853")
    assert sol.success
    return sol.y[0], sol.y[2]


def _peters_mathews_time(mc, f0, e0, freqs):
    return _peters_mathews(mc, f0, e0, freqs)[0]


def _oracle_cycles(m, mc, f0, e0, freqs):
    """GW cycles from f0 to f by the stationary-phase relation, from the
    oracle's phase Psi and time t: f t(f) - Psi(f)/2pi + Psi(f0)/2pi
    (t(f0) = 0 defines the coalescence time)."""
    fr, it, t, _ = O.phase(m, _theta(mc, f0, e0), np.concatenate([[f0], freqs]))
    psi = it + fr
    assert abs(t[0]) < 1e-6
    return freqs * t[1:] - psi[1:] + psi[0]


def test_time_follows_peters_mathews():
    """The eccentric shift of t(f) agrees with the integrated evolution to
    leading order: (oracle / ODE - 1) / e0^2 tends to a constant as e0 -> 0
    (the O(e0^4) remainder), which a wrong coefficient or exponent of the
    e0^2 term would turn into a non-vanishing offset."""
    mc, f0 = 28.0, 0.018
    freqs = f0 * np.array([1.05, 1.2, 1.5, 2.0, 3.0])
    m = _model(1)
    _, _, t_circ, _ = O.phase(m, _theta(mc, f0, 0.0), freqs)
    ode_circ = _peters_mathews_time(mc, f0, 0.0, freqs)
    # circular Newtonian chirp: the same to integration accuracy
    assert np.allclose(t_circ, ode_circ, rtol=1e-9, atol=0)
    scaled = []
    for e0 in (0.005, 0.01, 0.02, 0.05):
        _, _, t_ecc, _ = O.phase(m, _theta(mc, f0, e0), freqs)
        d_or = t_ecc - t_circ
        d_ode = _peters_mathews_time(mc, f0, e0, freqs) - ode_circ
        assert np.all(np.sign(d_or) == np.sign(d_ode)) and np.all(np.abs(d_ode) > 0)
        rel = d_or / d_ode - 1
        print(f"e0={e0}: eccentric time shift {d_ode} s, (oracle / ODE - 1) / e0^2 = {rel / e0 ** 2}")
        scaled.append(rel / e0 ** 2)
    scaled = np.array(scaled)
    assert np.all(np.abs(scaled) < 5.0)
    assert np.allclose(scaled[0], scaled[1], rtol=1e-3) and np.allclose(scaled[1], scaled[2], rtol=2e-3)


def test_phase_follows_peters_mathews():
    """The eccentric shift of the GW cycle count, formed from the oracle's
    phase by the stationary-phase relation, agrees with the cycles the
    Peters-Mathews evolution integrates, to leading order in e0^2:
    (oracle / ODE - 1) / e0^2 tends to a constant as e0 -> 0 (the O(e0^4)
    remainder).  The time shift is pinned on its own above, so a wrong
    coefficient or exponent in the eccentric phase term alone (which moves
    the cycle count by that term's change, hundreds of cycles here) fails
    this check; a relative error of 1e-3 in the term would read about -40 at
    e0 = 0.005."""
    mc, f0 = 28.0, 0.018
    freqs = f0 * np.array([1.05, 1.2, 1.5, 2.0, 3.0])
    m = _model(1)
    c_circ = _oracle_cycles(m, mc, f0, 0.0, freqs)
    _, ode_circ = _peters_mathews(mc, f0, 0.0, freqs)
    # circular Newtonian cycle count: the same to integration accuracy
    assert np.allclose(c_circ, ode_circ, rtol=1e-10, atol=0)
    scaled = []
    for e0 in (0.005, 0.01, 0.02, 0.05):
        d_or = _oracle_cycles(m, mc, f0, e0, freqs) - c_circ
        d_ode = _peters_mathews(mc, f0, e0, freqs)[1] - ode_circ
        assert np.all(np.sign(d_or) == np.sign(d_ode)) and np.all(np.abs(d_ode) > 10.0)
        rel = d_or / d_ode - 1
        print(f"e0={e0}: eccentric cycle shift {d_ode}, (oracle / ODE - 1) / e0^2 = {rel / e0 ** 2}")
        scaled.append(rel / e0 ** 2)
    scaled = np.array(scaled)
    assert np.all(np.abs(scaled) < 5.0)
    assert np.allclose(scaled[0], scaled[1], rtol=1e-3) and np.allclose(scaled[1], scaled[2], rtol=2e-3)


@pytest.mark.parametrize("e0", [0.05, 0.1])
def test_eccentric_time_is_phase_derivative(e0):
    """t(f) = (1/2pi) dPsi/df on the eccentric model at 3.5PN: the phase
    difference over a band equals the Gauss-Legendre integral of the oracle's
    time, so the separately written eccentric terms of phase and time agree
    (a factor off in either would leave a residual of order that term's
    share, seconds against the 1e-8-cycle check)."""
    import synth

    th = np.concatenate([synth.GW150914_LIKE, [e0]])
    m = O.Model(pn_order=7, eccentric=1)
    x, w = np.polynomial.legendre.leggauss(24)
    for f1, f2 in ((0.0181, 0.0186), (0.02, 0.0205), (0.024, 0.0245)):
        fr, it, _, _ = O.phase(m, th, [f1, f2])
        dphi = (it[1] - it[0]) + (fr[1] - fr[0])
        fq = 0.5 * (f2 - f1) * x + 0.5 * (f1 + f2)
        t = O.phase(m, th, fq)[2]
        integral = 0.5 * (f2 - f1) * np.sum(w * t)
        assert abs(dphi - integral) < 1e-8, (f1, dphi - integral)


def test_zero_eccentricity_is_the_circular_model():
    ds = D.lisa_small(seed=51)
    th7 = D.lisa_particles(6, seed=52)
    th7[0] = ds.injection
    th8 = np.concatenate([th7, np.zeros((6, 1))], axis=1)
    me = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=ds.model.t_obs, eccentric=1)
    a = O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, th7, 8, O.SEG_EQUAL_SNR, 16)["ups"]
    b = O.evaluate(ds.grid, me, ds.d_ri, ds.psd, th8, 8, O.SEG_EQUAL_SNR, 16)["ups"]
    assert np.array_equal(a, b)


def test_eccentric_injection_and_mismatch():
    """An eccentric injection is recovered exactly by the eccentric template
    (Upsilon_N = rho^2 for every N) and not by the circular one."""
    g = D.lisa_small(noise=False).grid
    me = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=1.0 / g.df, eccentric=1)
    f = (g.k0 + np.arange(g.K)) * g.df
    import synth

    s = 1.5 * synth.lisa_pn(f)
    psd = np.stack([s, s])
    inj = np.concatenate([synth.GW150914_LIKE, [0.1]])
    ds = D.make(g, me, psd, inj, 17.0, seed=0, noise=False)
    for N in (1, 16):
        u = O.evaluate(g, me, ds.d_ri, psd, inj[None, :], N, O.SEG_EQUAL_SNR, 16)["ups"][0]
        assert abs(u / 289.0 - 1) < 1e-12
    circ = inj.copy()
    circ[7] = 0.0
    u0 = O.evaluate(g, me, ds.d_ri, psd, circ[None, :], 1, O.SEG_EQUAL_SNR, 16)["ups"][0]
    print("circular template on the e0 = 0.1 injection: Upsilon_1 =", u0)
    assert u0 < 0.9 * 289.0


def test_invalid_eccentricity():
    ds = D.lisa_small(seed=53)
    me = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=ds.model.t_obs, eccentric=1)
    th = np.tile(np.concatenate([ds.injection, [0.01]]), (3, 1))
    th[1, 7] = -0.01
    th[2, 7] = 0.5
    u = O.evaluate(ds.grid, me, ds.d_ri, ds.psd, th, 4, O.SEG_EQUAL_SNR, 16)["ups"]
    assert np.isfinite(u[0]) and np.isnan(u[1]) and np.isnan(u[2])
