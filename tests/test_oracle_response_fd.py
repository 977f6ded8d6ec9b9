"""Pins of the oracle's full frequency-domain LISA response (response 2,
Sec 4 response paragraph: TDI transfer functions A, E, T).

1. Time-domain brute force: a monochromatic plane wave through the light-
   travel formula of every link, evaluated with explicit delays, then the
   first-generation TDI combination written with explicit delays (no
   factorisation, no sinc), against the oracle's closed form.  For a
   monochromatic wave and a frozen constellation the closed form is exact,
   so the two agree to rounding.
2. Low-frequency limit: A and E tend to the (separately pinned) low-frequency
   response at rate O(f L); T vanishes as (f L)^3.
3. Polarisation: psi -> psi + pi/2 flips the sign of every channel.
"""
import math

import numpy as np
import pytest

import oracle as O

C = 299792458.0
L = 2.5e9 / C  # light time of one arm [s]
YEAR = 31557600.0

MODEL_FD = O.Model(pn_order=7, response=O.RESP_LISA_FD, support=1, t_obs=6e7, orbit_phase0=0.3,
                   cartwheel_phase0=-1.1)
MODEL_LF = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=1, t_obs=6e7, orbit_phase0=0.3,
                   cartwheel_phase0=-1.1)


def _source(th):
    """Direction to the source, polarisation tensors and amplitudes of the
    template's (2,2) content: P = a+ e+ - i ax ex."""
    lam, bet, iota, psi = th[3], th[4], th[5], th[6]
    n = np.array([math.cos(bet) * math.cos(lam), math.cos(bet) * math.sin(lam), math.sin(bet)])
    u = np.array([math.sin(bet) * math.cos(lam), math.sin(bet) * math.sin(lam), -math.cos(bet)])
    v = np.array([math.sin(lam), -math.cos(lam), 0.0])
    p = math.cos(psi) * u + math.sin(psi) * v
    q = -math.sin(psi) * u + math.cos(psi) * v
    ep = np.outer(p, p) - np.outer(q, q)
    ex = np.outer(p, q) + np.outer(q, p)
    ap, ax = 0.5 * (1 + math.cos(iota) ** 2), math.cos(iota)
    return n, ap * ep - 1j * ax * ex


def _craft(t, model):
    """Spacecraft positions [3][3] in light-seconds relative to the centre:
    a rigid triangle in a plane inclined by 60 degrees, turning once a year."""
    Phi = model.orbit_phase0 + 2 * math.pi * t / YEAR
    er = np.array([math.cos(Phi), math.sin(Phi), 0.0])
    ephi = np.array([-math.sin(Phi), math.cos(Phi), 0.0])
    e1 = -0.5 * er - math.sqrt(3) / 2 * np.array([0.0, 0.0, 1.0])
    zeta = model.cartwheel_phase0 - Phi
    r = L / math.sqrt(3)
    return np.array([r * (math.cos(zeta + 2 * math.pi * a / 3) * e1 + math.sin(zeta + 2 * math.pi * a / 3) * ephi)
                     for a in range(3)])


def _tdi_time_domain(f, th, t0, model):
    """A, E, T of the wave P e^{2 pi i f t} (k = -nhat) at time t0, from
    y_ij(t) = n.[H(t - L - k.x_j) - H(t - k.x_i)].n / (2 (1 - k.n)) and
    X(t) = y01(t) + y10(t-L) + y02(t-2L) + y20(t-3L) - y02(t) - y20(t-L) - y01(t-2L) - y10(t-3L),
    the constellation frozen at t0; divided by the wave at t0 and by 4 (2 pi f L)^2."""
    nhat, P = _source(th)
    k = -nhat
    x = _craft(t0, model)

    def H(t):
        return P * np.exp(2j * math.pi * f * t)

    def y(i, j, t):
        n = (x[i] - x[j]) / L
        kn = k @ n
        return n @ (H(t - L - k @ x[j]) - H(t - k @ x[i])) @ n / (2 * (1 - kn))

    def michelson(a, b, c, t):
        return (y(a, b, t) + y(b, a, t - L) + y(a, c, t - 2 * L) + y(c, a, t - 3 * L)
                - y(a, c, t) - y(c, a, t - L) - y(a, b, t - 2 * L) - y(b, a, t - 3 * L))

    # the wave's phase is counted from t0 (a common factor), so the delays
    # are small arguments and the differences keep their precision
    X, Y, Z = michelson(0, 1, 2, 0.0), michelson(1, 2, 0, 0.0), michelson(2, 0, 1, 0.0)
    norm = 4 * (2 * math.pi * f * L) ** 2
    return np.array([(Z - X) / math.sqrt(2), (X - 2 * Y + Z) / math.sqrt(6), (X + Y + Z) / math.sqrt(3)]) / norm


def _thetas(n, seed):
    rng = np.random.default_rng(seed)
    th = np.zeros((n, 7))
    th[:, 0], th[:, 1], th[:, 2] = 28.0, 0.24, 0.018
    th[:, 3] = rng.uniform(0, 2 * math.pi, n)
    th[:, 4] = np.arcsin(rng.uniform(-1, 1, n))
    th[:, 5] = np.arccos(rng.uniform(-1, 1, n))
    th[:, 6] = rng.uniform(-math.pi, 0, n)
    return th


def test_geometry_of_the_check_matches_the_low_frequency_response():
    """The check's geometry and polarisation content reproduce the oracle's
    (pinned) low-frequency antenna patterns: D_X = (a01 a01 - a02 a02)/2 etc."""
    for th in _thetas(5, 1):
        for t in (0.0, 2.3e7):
            nhat, P = _source(th)
            x = _craft(t, MODEL_LF)
            arm = lambda a, b: (x[b] - x[a]) / L  # noqa: E731
            D = [0.5 * (np.outer(arm(a, b), arm(a, b)) - np.outer(arm(a, c), arm(a, c)))
                 for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1))]
            RA = np.sum((D[2] - D[0]) / math.sqrt(2) * P)
            RE = np.sum((D[0] - 2 * D[1] + D[2]) / math.sqrt(6) * P)
            F, _, _ = O.response(MODEL_LF, th, t)
            ap, ax = 0.5 * (1 + math.cos(th[5]) ** 2), math.cos(th[5])
            want = F[:, 0] * ap - 1j * F[:, 1] * ax
            assert np.allclose([RA, RE], want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("f", [3e-4, 4e-3, 0.016, 0.024, 0.032, 0.08])
def test_closed_form_equals_time_domain_delays(f):
    for th in _thetas(6, 2):
        for t in (0.0, 1.1e7, 4.4e7):
            got = O.fd_transfer(MODEL_FD, th, f, t)
            want = _tdi_time_domain(f, th, t, MODEL_FD)
            scale = np.abs(want[:2]).max()
            assert np.abs(got - want).max() < 1e-11 * scale, (f, t, got, want)


def test_low_frequency_limit():
    th_all = _thetas(8, 3)
    for th in th_all:
        for t in (0.0, 1.7e7):
            F, _, _ = O.response(MODEL_LF, th, t)
            ap, ax = 0.5 * (1 + math.cos(th[5]) ** 2), math.cos(th[5])
            lf = F[:, 0] * ap - 1j * F[:, 1] * ax
            errs, tch = [], []
            for f in (1e-6, 1e-5, 1e-4):
                x = 2 * math.pi * f * L
                R = O.fd_transfer(MODEL_FD, th, f, t)
                errs.append(np.abs(R[:2] - lf).max() / np.abs(lf).max() / x)
                tch.append(abs(R[2]) / np.abs(lf).max() / x ** 3)
            # first order in f L: the error over x settles to a constant, bounded by 4
            assert errs[-1] < 4.0 and abs(errs[0] / errs[1] - 1) < 1e-3 and abs(errs[1] / errs[2] - 1) < 1e-2
            # T: third order (at 1e-6 Hz T is rounding-limited, so compare the other two)
            assert tch[-1] < 4.0 and abs(tch[1] / tch[2] - 1) < 1e-2


def test_polarisation_quarter_turn_flips_sign():
    for th in _thetas(4, 4):
        th2 = th.copy()
        th2[6] += math.pi / 2
        for f in (0.017, 0.03):
            a = O.fd_transfer(MODEL_FD, th, f, 9e6)
            b = O.fd_transfer(MODEL_FD, th2, f, 9e6)
            assert np.allclose(a, -b, rtol=0, atol=1e-14 * np.abs(a).max())


def test_tdi_noise_psds_from_the_noise_sources():
    """The generator's A/E/T noise PSDs against the noise transfer of the same
    TDI combination computed source by source: link j -> i carries its own
    optical-metrology noise and the acceleration noise of both of its test
    masses (the one at j facing i, delayed by one arm, and the one at i facing
    j); every source independent.  Both in the full response's normalisation."""
    import synth

    c = 299792458.0
    f = np.array([1e-4, 1e-3, 0.01, 0.016, 0.024, 0.032, 0.05])
    s_oms, s_acc = 15e-12, 3e-15
    oms = s_oms ** 2 * (2 * math.pi * f / c) ** 2 * (1.0 + (2e-3 / f) ** 4)
    acc = s_acc ** 2 / (2 * math.pi * f * c) ** 2 * (1.0 + (0.4e-3 / f) ** 2) * (1.0 + (f / 8e-3) ** 4)
    z = np.exp(-2j * math.pi * f * L)
    links = [(i, j) for i in range(3) for j in range(3) if i != j]

    def tdi(coef):  # coef[(i, j)] = complex weight of link i <- j in y_ij, per frequency
        w = 1 - z ** 2

        def mich(a, b, cc):
            return w * ((coef[(a, b)] + z * coef[(b, a)]) - (coef[(a, cc)] + z * coef[(cc, a)]))

        X, Y, Z = mich(0, 1, 2), mich(1, 2, 0), mich(2, 0, 1)
        return np.array([(Z - X) / math.sqrt(2), (X - 2 * Y + Z) / math.sqrt(6), (X + Y + Z) / math.sqrt(3)])

    total = np.zeros((3, f.size))
    for src in links:  # optical-metrology noise of link src
        coef = {lk: (np.ones_like(z) if lk == src else np.zeros_like(z)) for lk in links}
        total += np.abs(tdi(coef)) ** 2 * oms
    for (i, j) in links:  # test mass at i facing j: in y_ij directly, in y_ji one arm later
        coef = {lk: np.zeros_like(z) for lk in links}
        coef[(i, j)] = coef[(i, j)] + 1.0
        coef[(j, i)] = coef[(j, i)] + z
        total += np.abs(tdi(coef)) ** 2 * acc
    x = 2 * math.pi * f * L
    want = total / (16 * x ** 4)
    got = synth.lisa_tdi_psd(f)
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    # low frequencies: A and E tend to 1.5 P_n
    lo = np.array([1e-5, 3e-5])
    assert np.allclose(synth.lisa_tdi_psd(lo)[0], 1.5 * synth.lisa_pn(lo), rtol=1e-6)
