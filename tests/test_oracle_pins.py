"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the fact it checks and where it comes from.  None of them
re-types the oracle's own formula: they use closed forms, invariants, special
cases that reduce to a textbook result, brute force on tiny inputs and values
printed in the paper.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import special

import oracle as O
import synth
from tests import datasets as D

GOLD = os.path.join(os.path.dirname(__file__), "golden")
T_SUN = 1.32712440018e20 / 299792458.0 ** 3
YEAR = 31557600.0


def _ups(ds, theta, N, mode=O.SEG_EQUAL_SNR, G=1, edges=None, **kw):
    return O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, np.atleast_2d(theta), N, mode, G, edges, **kw)


# ---------------------------------------------------------------- inner product

def test_hh_equals_hurwitz_zeta():
    """<h|h> for h = f^-7/6 in unit white noise is 4 df sum_k f_k^-7/3
    = 4 df^-4/3 [zeta(7/3, k0) - zeta(7/3, k0 + K)] (Hurwitz zeta), eqn:inner_prod
    discretised on the FFT grid."""
    ds = D.white_small(K=4096, noise=False, snr=0.0)
    out = _ups(ds, ds.injection, 1, want_seg=True)
    H = out["seg"][0, 0, 2]
    g = ds.grid
    exact = g.df ** (-7.0 / 3.0) * (special.zeta(7.0 / 3.0, g.k0) - special.zeta(7.0 / 3.0, g.k0 + g.K))
    assert abs(H / exact - 1.0) < 1e-12


def test_hh_continuum_limit():
    """The same sum approaches the integral (3/4) (f0^-4/3 - fK^-4/3) / df to O(df)."""
    ds = D.white_small(K=4096, noise=False, snr=0.0)
    H = _ups(ds, ds.injection, 1, want_seg=True)["seg"][0, 0, 2]
    g = ds.grid
    f0, fK = g.k0 * g.df, (g.k0 + g.K) * g.df
    integral = 0.75 * (f0 ** (-4 / 3) - fK ** (-4 / 3)) / g.df
    assert abs(H / integral - 1.0) < 2.0 * g.K ** -1


# ---------------------------------------------------------------- boundaries

def test_equal_snr_boundaries_power_law():
    """White noise, no response: w ~ f^-7/3, so equal [h|h] segments have
    continuous edges f_n = [f0^-4/3 - (n/N)(f0^-4/3 - fK^-4/3)]^-3/4 (Sec 2.2,
    boundary choice); the discrete rule lands within one bin of them."""
    ds = D.white_small(K=4096, noise=False, snr=0.0)
    g = ds.grid
    for N in (4, 16, 64):
        b = _ups(ds, ds.injection, N, want_bounds=True)["bounds"][0]
        f0, fK = g.k0 * g.df, (g.k0 + g.K) * g.df
        n = np.arange(N + 1)
        fn = (f0 ** (-4 / 3) - n / N * (f0 ** (-4 / 3) - fK ** (-4 / 3))) ** (-0.75)
        kn = fn / g.df - g.k0
        assert b[0] == 0 and b[-1] == g.K
        assert np.all(np.abs(b - kn) <= 1.0 + 1e-9), (N, b - kn)


def test_equal_snr_boundaries_brute_force_dense():
    """G = 1 rule against a brute-force cumulative over the oracle's own
    template weights (tiny input)."""
    ds = D.white_small(K=512, noise=False, snr=0.0)
    h = O.template(ds.grid, ds.model, ds.injection)
    w = np.abs(h[0]) ** 2
    C = np.concatenate([[0.0], np.cumsum(w)])
    for N in (3, 7, 16):
        b = _ups(ds, ds.injection, N, want_bounds=True)["bounds"][0]
        for n in range(1, N):
            target = n / N * C[-1]
            k = int(np.argmax(C >= target))
            assert abs(b[n] - k) <= 0, (N, n, b[n], k)


def test_equal_snr_edges_two_nodes_closed_form():
    """Node stride G >= the support length: the rule's only nodes are k_lo and
    k_hi - 1, the weight is linear between them, the cumulative is the
    quadratic C(k_lo + m) = m w0 + d m(m - 1)/2 with d = (w1 - w0)/(L - 1),
    and the edges are its crossings of the targets (n/N) C(k_hi).  On the
    white one-channel model the weight is f^-7/3 (the template's |h|^2, up to
    a constant that the targets do not see), so the edges follow in exact
    rational arithmetic; the oracle sums the interpolated weights bin by bin
    in FP64 and may differ only where a target lies within its rounding."""
    from fractions import Fraction as Fr

    ds = D.white_small(K=600, noise=False, snr=0.0)
    g = ds.grid
    L = g.K
    f = lambda k: (g.k0 + k) * g.df  # noqa: E731
    w0, w1 = Fr(f(0) ** (-7.0 / 3.0)), Fr(f(L - 1) ** (-7.0 / 3.0))
    d = (w1 - w0) / (L - 1)
    C = lambda m: m * w0 + d * m * (m - 1) / 2  # noqa: E731
    tot = C(L)
    checked = 0
    for N in (3, 7, 16, 50):
        b = _ups(ds, ds.injection, N, G=4096, want_bounds=True)["bounds"][0]
        assert b[0] == 0 and b[-1] == L
        m = 0
        for n in range(1, N):
            tgt = Fr(n, N) * tot
            while C(m) < tgt:
                m += 1
            near = min(abs(C(m) - tgt), abs(C(m - 1) - tgt) if m > 0 else tgt) < Fr(1, 10 ** 12) * tot
            if not near:
                assert b[n] == m, (N, n, b[n], m)
                checked += 1
            else:
                assert abs(b[n] - m) <= 1
    assert checked >= 70
    # the interpolation matters: the dense rule (G = 1, the exact f^-7/3
    # weights) moves at least one of these edges
    assert not np.array_equal(_ups(ds, ds.injection, 50, G=1, want_bounds=True)["bounds"][0],
                              _ups(ds, ds.injection, 50, G=4096, want_bounds=True)["bounds"][0])


def test_one_bin_per_segment_gives_the_data_norm():
    """With one channel and one bin per segment, every term is
    4 df |d conj(h)/S|^2 / (|h|^2/S) = 4 df |d|^2/S (Sec 2.2, the statistic
    at its finest segmentation): Upsilon_N is <d|d> over the support whatever
    the template, so on the full-support white model it does not depend on
    Mc or eta at all."""
    ds = D.white_small(K=512, noise=True, snr=12.0)
    g = ds.grid
    dd = O.data_norm(g, ds.d_ri, ds.psd)
    th = np.tile(ds.injection, (4, 1))
    th[1, 0], th[2, 1], th[3, :2] = 25.0, 0.2, (34.0, 0.16)
    for mode, edges in ((O.SEG_UNIFORM, None), (O.SEG_EXPLICIT, np.arange(g.K + 1, dtype=np.int64))):
        u = _ups(ds, th, g.K, mode=mode, edges=edges)["ups"]
        assert np.allclose(u, dd, rtol=1e-12, atol=0), (mode, u, dd)
    # and at any coarser segmentation it is below <d|d> (Cauchy-Schwarz)
    assert np.all(_ups(ds, th, 64, mode=O.SEG_UNIFORM)["ups"] < dd)


def test_boundaries_nest_and_refinement_increases_upsilon():
    """For N | N' the equal-SNR targets nest, so the boundaries nest; splitting
    a segment can only raise sum |Z|^2/H (Cauchy-Schwarz), hence
    Upsilon_{N'} >= Upsilon_N (Sec 2.2)."""
    ds = D.lisa_small(seed=5)
    th = D.lisa_particles(6, seed=3)
    th[0] = ds.injection
    prev = None
    for N in (4, 8, 16, 32):
        out = _ups(ds, th, N, G=64, want_bounds=True)
        if prev is not None:
            pb, pu = prev
            assert np.all(out["bounds"][:, ::2] == pb)
            assert np.all(out["ups"] >= pu * (1 - 1e-13))
        prev = (out["bounds"], out["ups"])


def test_uniform_and_explicit_modes():
    ds = D.white_small(K=1000, noise=True)
    N = 7
    b = _ups(ds, ds.injection, N, mode=O.SEG_UNIFORM, want_bounds=True)["bounds"][0]
    assert list(b) == [n * 1000 // N for n in range(N + 1)]
    edges = np.array([0, 10, 10, 400, 999, 1000, 1000, 1000], dtype=np.int64)
    out = _ups(ds, ds.injection, N, mode=O.SEG_EXPLICIT, edges=edges, want_bounds=True, want_seg=True)
    assert list(out["bounds"][0]) == list(edges)
    # empty segments contribute exactly zero
    assert np.all(out["seg"][0, [1, 5, 6]] == 0.0)


# ---------------------------------------------------------------- statistic

def test_upsilon1_is_phase_maximised_matched_filter():
    """N = 1: Upsilon_1 = max_phi <d|h e^{i phi}>^2 / <h|h> (Sec 2.2: the
    square of the phase-maximised coherent statistic), by brute force over a
    fine phase grid using the oracle's template."""
    ds = D.white_small(K=2048, seed=4)
    th = ds.injection.copy()
    th[0] *= 1.0000003
    ups = _ups(ds, th, 1)["ups"][0]
    h = O.template(ds.grid, ds.model, th)
    hh = D.inner(ds.grid, ds.psd, h, h)
    phis = np.linspace(0, 2 * np.pi, 20001)
    z = np.sum(ds.d[0] * np.conj(h[0]) / ds.psd[0])
    x = 4 * ds.grid.df * np.real(np.exp(-1j * phis) * z)
    brute = np.max(x) ** 2 / hh
    assert abs(ups / brute - 1) < 1e-7


def test_noise_free_injection_gives_rho_squared():
    """d = h(theta*): every segment term equals [h|h]_n, so Upsilon_N = rho^2
    for every N and every segmentation."""
    for ds in (D.white_small(K=2048, noise=False, snr=20.0), D.lisa_small(noise=False, snr=17.0),
               D.lisa_small(noise=False, snr=17.0, response=O.RESP_LISA_FD),
               D.lisa_small(noise=False, snr=17.0, response=O.RESP_LISA_FD, n_chan=3)):
        for N in (1, 5, 32):
            for mode in (O.SEG_EQUAL_SNR, O.SEG_UNIFORM):
                u = _ups(ds, ds.injection, N, mode=mode, G=16)["ups"][0]
                assert abs(u / ds.snr ** 2 - 1) < 1e-12, (N, mode, u)


def test_scale_and_phase_invariance():
    """Upsilon is blind to the distance (1/D_L prefactor) and to a constant
    phase (Sec 4: D_L cancels; phase maximised), and scales as |c|^2 with the data."""
    ds = D.lisa_small(seed=8)
    th = D.lisa_particles(4, seed=9)
    th[0] = ds.injection
    base = _ups(ds, th, 16, G=32)["ups"]
    c = 0.37 * np.exp(1.1j)
    d2 = D.Dataset(ds.grid, ds.model, ds.psd, ds.d * c, ds.injection, ds.snr, ds.lo, ds.hi)
    scaled = _ups(d2, th, 16, G=32)["ups"]
    assert np.allclose(scaled, base * abs(c) ** 2, rtol=1e-12, atol=0)


@pytest.mark.parametrize("response,n_chan", [(O.RESP_LISA_LF_AE, 2), (O.RESP_LISA_FD, 2), (O.RESP_LISA_FD, 3)])
def test_polarisation_period_quarter_turn(response, n_chan):
    """psi -> psi + pi/2 flips the sign of both polarisation tensors, i.e. of
    the whole template, which the statistic cannot see."""
    ds = D.lisa_small(seed=12, response=response, n_chan=n_chan)
    th = D.lisa_particles(5, seed=13)
    th2 = th.copy()
    th2[:, 6] += np.pi / 2
    a = _ups(ds, th, 8, G=32)["ups"]
    b = _ups(ds, th2, 8, G=32)["ups"]
    assert np.allclose(a, b, rtol=1e-11, atol=0)


def test_full_response_t_channel_adds_its_own_terms():
    """With A, E and T the per-segment sums are those of A+E plus those of T
    alone (the channels add inside each segment at fixed edges)."""
    ds3 = D.lisa_small(seed=16, response=O.RESP_LISA_FD, n_chan=3)
    th = D.lisa_particles(4, seed=17)
    th[0] = ds3.injection
    edges = np.linspace(ds3.grid.K // 4, ds3.grid.K, 9).astype(np.int64)
    full = O.evaluate(ds3.grid, ds3.model, ds3.d_ri, ds3.psd, th, 8, O.SEG_EXPLICIT, 1, edges, want_seg=True)
    h = [O.template(ds3.grid, ds3.model, t) for t in th]
    for p in range(th.shape[0]):
        for n in range(8):
            sl = slice(max(edges[n], full["support"][p][0]), min(edges[n + 1], full["support"][p][1]))
            z = np.sum(ds3.d[:, sl] * np.conj(h[p][:, sl]) / ds3.psd[:, sl], axis=1)
            hh = np.sum(np.abs(h[p][:, sl]) ** 2 / ds3.psd[:, sl], axis=1)
            assert abs(complex(*full["seg"][p, n, :2]) - z.sum()) <= 1e-12 * np.sqrt(hh.sum() * np.sum(
                np.abs(ds3.d[:, sl]) ** 2 / ds3.psd[:, sl]))
            assert abs(full["seg"][p, n, 2] - hh.sum()) <= 1e-12 * hh.sum()


def test_cauchy_schwarz_bound():
    """Each term 4 df |Z_n|^2 / H_n <= [d|d]_n, so Upsilon_N <= <d|d> over the support."""
    ds = D.lisa_small(seed=14)
    th = D.lisa_particles(8, seed=15)
    out = _ups(ds, th, 64, G=16)
    for p in range(th.shape[0]):
        lo, hi = out["support"][p]
        dd = 4 * ds.grid.df * np.sum(np.abs(ds.d[:, lo:hi]) ** 2 / ds.psd[:, lo:hi])
        assert out["ups"][p] <= dd


def test_invalid_and_empty_support():
    ds = D.lisa_small(seed=2)
    th = np.tile(ds.injection, (4, 1))
    th[0, 0] = -1.0          # Mc <= 0
    th[1, 1] = 0.3           # eta > 1/4
    th[2, 2] = 0.0185        # f_low above the observation window of this band? keeps support
    th[3, 2] = 0.0195        # f_low above the band: empty support
    out = _ups(ds, th, 4, G=32)
    assert np.isnan(out["ups"][0]) and np.isnan(out["ups"][1])
    assert out["ups"][3] == 0.0


# ---------------------------------------------------------------- noise statistics

@pytest.mark.slow
@pytest.mark.parametrize("N", [1, 4, 10])
@pytest.mark.parametrize("snr", [0.0, 10.0])
def test_chi2_law_over_noise(N, snr):
    """At fixed theta and boundaries, each term is a non-central chi^2 with
    two degrees of freedom, so Upsilon_N ~ chi^2_{2N}(rho^2).  Its mean 2N + rho^2
    and variance 4N + 4 rho^2 are the moments of eqn:CLTdist_noise /
    eqn:CLTdist_signal with (mu_k, sigma_k) = (2, sqrt 2)."""
    from scipy import stats

    gold = json.load(open(os.path.join(GOLD, "paper_tables.json")))["clt_moments"]
    base = D.white_small(K=512, noise=False, snr=snr)
    h = base.d.copy()
    vals = []
    for s in range(800):
        n = synth.noise(base.psd, base.grid.df, 10_000 + s)
        ds = D.Dataset(base.grid, base.model, base.psd, h + n, base.injection, snr, None, None)
        vals.append(_ups(ds, base.injection, N, mode=O.SEG_UNIFORM)["ups"][0])
    vals = np.array(vals)
    p = stats.kstest(vals, stats.ncx2(2 * N, snr ** 2).cdf if snr > 0 else stats.chi2(2 * N).cdf).pvalue
    assert p > 1e-3
    mean = gold["mean_noise_per_segment"] * N + snr ** 2
    var = gold["var_noise_per_segment"] * N + gold["var_signal_extra_per_rho2"] * snr ** 2
    assert abs(vals.mean() - mean) < 4 * math.sqrt(var / len(vals))


@pytest.mark.slow
def test_normalisation_against_paper_best_values():
    """E[Upsilon_1(theta*)] = rho^2 + 2 with sd 2 sqrt(1 + rho^2); the paper's
    best Upsilon_1 values (Table tab:Best_upsilons, maxima over theta) sit
    within three standard deviations of it, which fixes the factor-4 and noise
    normalisation conventions."""
    gold = json.load(open(os.path.join(GOLD, "paper_tables.json")))["best_upsilon_1"]
    for snr in (38, 22, 20):
        base = D.white_small(K=256, noise=False, snr=float(snr))
        vals = []
        for s in range(300):
            n = synth.noise(base.psd, base.grid.df, 77_000 + s)
            ds = D.Dataset(base.grid, base.model, base.psd, base.d + n, base.injection, snr, None, None)
            vals.append(_ups(ds, base.injection, 1)["ups"][0])
        m = np.mean(vals)
        sd = 2 * math.sqrt(1 + snr ** 2)
        assert abs(m - (snr ** 2 + 2)) < 4 * sd / math.sqrt(len(vals))
        for v in gold[str(snr)]:
            assert abs(v - m) < 3 * sd


# ---------------------------------------------------------------- waveform

def test_newtonian_chirp_time_closed_form():
    """At Newtonian order t_c = tau(f_low) = (5/256) (pi f_low)^-8/3 (G Mc/c^3)^-5/3,
    the textbook chirp time, whatever eta is."""
    for mc, eta, fl in [(28.095555, 0.2471, 0.018), (95.0209, 0.234, 0.0175), (5.0, 0.1, 0.03)]:
        th = np.array([mc, eta, fl, 0, 0, 0, 0])
        tc = O.phase(O.Model(pn_order=0), th, [fl])[3]
        exact = 5.0 / 256.0 * (math.pi * fl) ** (-8 / 3) * (mc * T_SUN) ** (-5 / 3)
        assert abs(tc / exact - 1) < 1e-13


def test_newtonian_cycle_count_closed_form():
    """GW cycles between f1 and f2 at Newtonian order:
    N = (G Mc/c^3)^-5/3 (f1^-5/3 - f2^-5/3) / (32 pi^8/3).  From the SPA,
    the cycle count up to f is f t(f) - Psi(f)/2pi (+ const)."""
    mc, eta = 28.095555, 0.2471
    th = np.array([mc, eta, 0.018, 0, 0, 0, 0])
    f1, f2 = 0.0185, 0.0243
    fr, it, t, _ = O.phase(O.Model(pn_order=0), th, [f1, f2])
    Phi = it + fr
    cyc = (f2 * t[1] - Phi[1]) - (f1 * t[0] - Phi[0])
    exact = (mc * T_SUN) ** (-5 / 3) * (f1 ** (-5 / 3) - f2 ** (-5 / 3)) / (32 * math.pi ** (8 / 3))
    assert abs(cyc / exact - 1) < 1e-9


def test_spa_time_is_phase_derivative():
    """t(f) = (1/2pi) dPsi/df at 3.5PN (log terms included): the phase
    difference over a band equals the Gauss-Legendre integral of t(f).  The
    check resolves ~1e-5 s in t, well below the 3.5PN term (~1 s)."""
    th = synth.GW150914_LIKE
    m = O.Model(pn_order=7)
    x, w = np.polynomial.legendre.leggauss(24)
    for f1, f2 in ((0.0181, 0.0186), (0.02, 0.0205), (0.024, 0.0245)):
        fr, it, _, _ = O.phase(m, th, [f1, f2])
        dphi = (it[1] - it[0]) + (fr[1] - fr[0])
        fq = 0.5 * (f2 - f1) * x + 0.5 * (f1 + f2)
        t = O.phase(m, th, fq)[2]
        integral = 0.5 * (f2 - f1) * np.sum(w * t)
        assert abs(dphi - integral) < 1e-8, (f1, dphi - integral)


def test_phase_accuracy_against_mpmath():
    """Extended-precision phase against a 40-digit evaluation of the same
    series at sampled grid bins (rounding check, 1e-11 cycles)."""
    import mpmath as mp

    mp.mp.dps = 40
    th = synth.GW150914_LIKE
    eta, mc = mp.mpf(th[1]), mp.mpf(th[0])
    tsun = mp.mpf("1.32712440018e20") / mp.mpf(299792458) ** 3
    piM = mp.pi * mc * eta ** mp.mpf("-0.6") * tsun
    pref = 3 / (256 * mp.pi * eta)
    g = mp.euler
    psi = {0: 1, 2: mp.mpf(3715) / 756 + 55 * eta / 9, 3: -16 * mp.pi,
           4: mp.mpf(15293365) / 508032 + 27145 * eta / 504 + 3085 * eta ** 2 / 72,
           7: mp.pi * (mp.mpf(77096675) / 254016 + 378515 * eta / 1512 - 74045 * eta ** 2 / 756)}
    a5 = mp.pi * (mp.mpf(38645) / 756 - 65 * eta / 9)
    p6 = (mp.mpf(11583231236531) / 4694215680 - 640 * mp.pi ** 2 / 3 - 6848 * g / 21
          + (mp.mpf(-15737765635) / 3048192 + 2255 * mp.pi ** 2 / 12) * eta
          + 76055 * eta ** 2 / 1728 - 127825 * eta ** 3 / 1296)

    def series(v):
        s = 0
        for j in (0, 2, 3, 4, 7):
            s += psi[j] * v ** j
        s += a5 * (1 + 3 * mp.log(v * mp.sqrt(6))) * v ** 5
        s += (p6 - mp.mpf(6848) / 21 * mp.log(4 * v)) * v ** 6
        return s / v ** 5

    def dseries(v):  # f d/df series
        return mp.diff(lambda x: series(x), v) * v / 3

    fl = mp.mpf(th[2])
    tc = -pref * dseries(mp.cbrt(piM * fl)) / fl
    spec = synth.GridSpec(1 << 20)
    grid = O.Grid(spec.K, spec.k0, spec.df, 2)
    bins = np.array([131072, 200001, 333333, 500000, 777777])
    fr, _ = O.phase_bins(grid, O.Model(pn_order=7), th, bins)
    for b, x in zip(bins, fr):
        f = mp.mpf(int(spec.k0 + b)) * mp.mpf(spec.df)
        ph = f * tc - mp.mpf(1) / 8 + pref * series(mp.cbrt(piM * f))
        ref = float(ph - mp.floor(ph))
        d = abs(ref - x)
        d = min(d, 1 - d)
        assert d < 1e-11, (b, d)


def test_coalescence_time_matches_paper_tables():
    """t_c derived from f_low is listed in the injection tables (43.28 and 6.12
    months, TaylorF2Ecc with e0 = 0.01, 0.03); the circular 3.5PN model lands
    within 3%.  The tables' (m1, m2) also reproduce the listed (Mc, eta)."""
    gold = json.load(open(os.path.join(GOLD, "paper_tables.json")))
    for key in ("gw150914_like", "gw190521_like"):
        src = gold[key]
        th = np.array([src["Mc"], src["eta"], src["f_low"], 0, 0, 0, 0])
        tc = O.phase(O.Model(pn_order=7), th, [src["f_low"]])[3]
        months = tc / (YEAR / 12)
        assert abs(months / src["tc_months"] - 1) < 0.03, (key, months)
        m1, m2 = src["m1"], src["m2"]
        mc = (m1 * m2) ** 0.6 / (m1 + m2) ** 0.2
        eta = m1 * m2 / (m1 + m2) ** 2
        assert abs(mc / src["Mc"] - 1) < 2e-3 and abs(eta - src["eta"]) < 1e-3


def test_support_edges():
    """Observation window: the first bin at or above f_low (exact rational
    arithmetic), and the last bin whose SPA time is below T_obs."""
    ds = D.lisa_small(noise=False)
    th = D.lisa_particles(5, seed=31)
    out = _ups(ds, th, 2, G=64)
    g = ds.grid
    for p in range(th.shape[0]):
        lo, hi = out["support"][p]
        k = 0
        df = Fraction(g.df)
        fl = Fraction(th[p, 2])
        kk = math.ceil(fl / df) - g.k0
        assert lo == max(0, kk)
        _, t = O.phase_bins(g, ds.model, th[p], np.array([hi - 1, hi]))
        assert t[0] < ds.model.t_obs <= t[1]


# ---------------------------------------------------------------- response

def _rand_sky(rng, n):
    lam = rng.uniform(0, 2 * np.pi, n)
    beta = np.arcsin(rng.uniform(-1, 1, n))
    psi = rng.uniform(-np.pi, 0, n)
    iota = np.arccos(rng.uniform(-1, 1, n))
    return lam, beta, psi, iota


def test_response_ae_sum_closed_form():
    """A and E are orthogonal, equal-norm, traceless tensors in the detector
    plane (|D_A|^2 = |D_E|^2 = 9/16 for a 60-degree triangle), so
    sum_{A,E} (F+^2 + Fx^2) = (9/8) [(1 + c^2)^2 / 4 + c^2] with c the cosine
    between the source direction and the plane normal z/2 - (sqrt3/2) r_hat(t)
    (plane inclined 60 degrees to the ecliptic)."""
    rng = np.random.default_rng(0)
    m = O.Model()
    lam, beta, psi, iota = _rand_sky(rng, 200)
    ts = rng.uniform(0, 3 * YEAR, 200)
    for i in range(200):
        th = np.array([28.0, 0.24, 0.018, lam[i], beta[i], iota[i], psi[i]])
        F, dop, tch = O.response(m, th, ts[i])
        Phi = 2 * np.pi * ts[i] / YEAR
        nd = np.array([-np.sqrt(3) / 2 * np.cos(Phi), -np.sqrt(3) / 2 * np.sin(Phi), 0.5])
        n = np.array([np.cos(beta[i]) * np.cos(lam[i]), np.cos(beta[i]) * np.sin(lam[i]), np.sin(beta[i])])
        c = n @ nd
        expect = 9 / 8 * ((1 + c * c) ** 2 / 4 + c * c)
        assert abs(np.sum(F ** 2) - expect) < 1e-12
        assert np.all(np.abs(tch) < 1e-14)  # T = (X + Y + Z)/sqrt3 has no response


def test_response_sky_average():
    """Sky- and polarisation-averaged F+^2 + Fx^2 = (4/5)|D|^2 for a traceless
    detector tensor: 9/20 for A and for E; A-E cross term averages to 0."""
    rng = np.random.default_rng(1)
    m = O.Model()
    n = 20000
    lam, beta, psi, iota = _rand_sky(rng, n)
    acc = np.zeros(3)
    for i in range(n):
        th = np.array([28.0, 0.24, 0.018, lam[i], beta[i], iota[i], psi[i]])
        F, _, _ = O.response(m, th, 1.234e6)
        acc += [F[0] @ F[0], F[1] @ F[1], F[0] @ F[1]]
    acc /= n
    assert abs(acc[0] - 0.45) < 0.01 and abs(acc[1] - 0.45) < 0.01 and abs(acc[2]) < 0.01


def test_doppler_sign_and_light_travel_time():
    """Source in the ecliptic at the constellation's longitude: the detector
    is 1 AU closer, the signal arrives earlier by AU/c = 499.005 s, and the
    Doppler phase per Hz is -AU/c (template ~ e^{-i 2 pi (Psi + Phi_D)})."""
    m = O.Model()
    t = 0.3 * YEAR
    lam = 2 * np.pi * 0.3
    _, dop, _ = O.response(m, np.array([28.0, 0.24, 0.018, lam, 0.0, 1.0, -1.0]), t)
    assert abs(dop + 1.495978707e11 / 299792458.0) < 1e-9
    _, dop, _ = O.response(m, np.array([28.0, 0.24, 0.018, lam, np.pi / 2, 1.0, -1.0]), t)
    assert abs(dop) < 1e-9


# ---------------------------------------------------------------- PSO and RNG

def test_philox_known_answers():
    kat = json.load(open(os.path.join(GOLD, "philox_kat.json")))["vectors"]
    for v in kat:
        out = O.philox4x32_10([int(x, 16) for x in v["ctr"]], [int(x, 16) for x in v["key"]])
        assert out == [int(x, 16) for x in v["out"]]


def test_uniform_range_and_moments():
    u = np.array([O.uniform(123, 0, 1, p, d, 0) for p in range(2000) for d in range(3)])
    assert np.all(u > 0) and np.all(u < 1)
    assert abs(u.mean() - 0.5) < 0.02 and abs(u.var() - 1 / 12) < 0.01


def test_pso_move_hand_computed():
    """eqn:PSO_velocity_rule then eqn:PSO_min_velocity, one particle, two
    dimensions, worked by hand from the drawn uniforms."""
    seed, swarm, it = 99, 3, 7
    th = np.array([[1.0, 2.0]])
    v = np.array([[0.1, -0.001]])
    pb = np.array([[2.0, 2.5]])
    gb = np.array([-1.0, 2.0])
    lo, hi = np.array([-10.0, -10.0]), np.array([10.0, 10.0])
    eps = np.array([0.0, 0.05])
    O.pso_move(th, v, pb, gb, 0.5, 0.2, 0.3, eps, lo, hi, [0, 0], seed, swarm, it)
    rp0, rg0 = O.uniform(seed, swarm, it, 0, 0, 0), O.uniform(seed, swarm, it, 0, 0, 1)
    rp1, rg1 = O.uniform(seed, swarm, it, 0, 1, 0), O.uniform(seed, swarm, it, 0, 1, 1)
    u0 = 0.05 + 0.2 * rp0 * 1.0 + 0.3 * rg0 * (-2.0)
    u1 = -0.0005 + 0.2 * rp1 * 0.5 + 0.3 * rg1 * 0.0
    v1 = u1 if abs(u1) >= 0.05 else math.copysign(0.05, u1)
    assert abs(v[0, 0] - u0) < 1e-15 and abs(th[0, 0] - (1.0 + u0)) < 1e-15
    assert abs(v[0, 1] - v1) < 1e-15 and abs(th[0, 1] - (2.0 + v1)) < 1e-15
    assert abs(v[0, 1]) >= 0.05


def test_pso_periodic_wrap_and_min_velocity():
    rng = np.random.default_rng(5)
    P, Dm = 200, 7
    lo, hi = synth.GW150914_PRIOR_LO, synth.GW150914_PRIOR_HI
    th = O.pso_init(P, lo, hi, 42, 0)
    assert np.all(th >= lo) and np.all(th <= hi)
    v = rng.normal(size=(P, Dm)) * (hi - lo) * 0.3
    pb = O.pso_init(P, lo, hi, 43, 0)
    gb = pb[0].copy()
    eps = np.array([0.1, 0.05, 5e-8, 0.1, 0.1, 0.2, 0.1])
    O.pso_move(th, v, pb, gb, 0.5, 0.2, 0.3, eps, lo, hi, synth.PERIODIC, 42, 0, 1)
    assert np.all(np.abs(v) >= eps)
    for d in (3, 6):
        assert np.all(th[:, d] >= lo[d]) and np.all(th[:, d] < hi[d])


def test_pso_best_update():
    lo, hi = np.zeros(2), np.ones(2)
    th = np.array([[0.5, 0.5], [0.2, 1.5], [0.1, 0.1], [0.9, 0.9]])
    vals = np.array([3.0, 100.0, np.nan, 3.0])
    pb = np.zeros_like(th)
    pbv = np.array([2.0, 1.0, 1.0, 5.0])
    gb = np.zeros(2)
    g = O.pso_best(th, vals, lo, hi, [0, 0], pb, pbv, gb, 4.0)
    # particle 1 is out of the box, particle 2 NaN: neither moves
    assert list(pbv) == [3.0, 1.0, 1.0, 5.0]
    assert np.all(pb[0] == th[0]) and np.all(pb[1] == 0)
    assert g == 5.0 and np.all(gb == pb[3])


@pytest.mark.slow
def test_chi2_law_two_channels_share_phase():
    """A+E: the phase e^{i phi_n} multiplies h before the channel sum (Sec 2.2
    segmented product), so each segment keeps two degrees of freedom and
    Upsilon_N ~ chi^2_{2N}(rho^2), not chi^2_{4N}."""
    from scipy import stats

    base = D.lisa_small(K=8000, f_min=0.0179, noise=False, snr=8.0)
    vals = []
    for s in range(300):
        n = synth.noise(base.psd, base.grid.df, 30_000 + s)
        ds = D.Dataset(base.grid, base.model, base.psd, base.d + n, base.injection, base.snr, None, None)
        vals.append(_ups(ds, base.injection, 4, mode=O.SEG_UNIFORM)["ups"][0])
    p = stats.kstest(np.array(vals), stats.ncx2(8, base.snr ** 2).cdf).pvalue
    assert p > 1e-3


# ---------------------------------------------------------------- likelihoods (Sec 2.1 - 2.2)
def _stats(ds, theta, N, mode=O.SEG_EQUAL_SNR, G=1, edges=None):
    return O.likelihood_stats(ds.grid, ds.model, ds.d_ri, ds.psd, np.atleast_2d(theta), N, mode, G, edges)


def test_likelihood_noise_free_injection_is_zero():
    """d = A h(theta*): <d|d> = A^2 <h|h>, and at the true amplitude and phase
    the coherent log L (eqn:LogL_coherent) and, for every N, the semi-coherent
    log hat L_N are exactly zero (d - A h = 0; every segment's phase is already
    right).  <h|h> against a direct sum over the template's bins."""
    for ds in (D.white_small(K=2048, noise=False, snr=20.0), D.lisa_small(noise=False, snr=17.0),
               D.lisa_small(noise=False, snr=17.0, response=O.RESP_LISA_FD),
               D.lisa_small(noise=False, snr=17.0, response=O.RESP_LISA_FD, n_chan=3)):
        h = O.template(ds.grid, ds.model, ds.injection)
        hh_bf = D.inner(ds.grid, ds.psd, h, h)
        amp = ds.snr / math.sqrt(hh_bf)
        dd = O.data_norm(ds.grid, ds.d_ri, ds.psd)
        assert abs(dd / (amp ** 2 * hh_bf) - 1) < 1e-12
        for N in (1, 5, 32):
            st = _stats(ds, ds.injection, N, G=16)
            assert abs(st["hh"][0] / hh_bf - 1) < 1e-12
            semi, coh = O.loglike(dd, st, amp, phase=0.0)
            assert abs(semi[0]) < 1e-10 * dd and abs(coh[0]) < 1e-10 * dd, (N, semi, coh)


def test_likelihood_phase_convention():
    """With d = A h e^{i phi0}, <d|h e^{i phi}> = A <h|h> cos(phi - phi0)
    (eqn:inner_prod: the second argument is conjugated), so the coherent log L
    is zero at phi = phi0 and below zero at -phi0."""
    ds = D.lisa_small(noise=False, snr=17.0)
    phi0 = 0.7
    d = ds.d * np.exp(1j * phi0)
    d_ri = np.stack([d.real, d.imag], -1)
    st = O.likelihood_stats(ds.grid, ds.model, d_ri, ds.psd, np.atleast_2d(ds.injection), 8, O.SEG_EQUAL_SNR, 1)
    assert abs(np.angle(st["dh"][0]) - phi0) < 1e-12
    dd = O.data_norm(ds.grid, d_ri, ds.psd)
    amp = ds.snr / math.sqrt(st["hh"][0])
    _, coh = O.loglike(dd, st, amp, phase=phi0)
    _, coh_neg = O.loglike(dd, st, amp, phase=-phi0)
    assert abs(coh[0]) < 1e-10 * dd
    assert coh_neg[0] < -0.1 * dd


def test_likelihood_inner_products_against_direct_sums():
    """On noisy data and off-peak particles, <h|h> and the complex <d|h> equal
    4 df sum_k d conj(h) / S summed directly over the template's bins (which
    vanish outside the support), for any segmentation; Upsilon_1 = |<d|h>|^2/<h|h>."""
    ds = D.lisa_small(seed=12)
    th = D.lisa_particles(3, seed=41)
    th[0] = ds.injection
    for p in range(th.shape[0]):
        h = O.template(ds.grid, ds.model, th[p])
        hh = D.inner(ds.grid, ds.psd, h, h)
        dh = 4.0 * ds.grid.df * np.sum(ds.d * np.conj(h) / ds.psd)
        for N in (1, 16):
            st = _stats(ds, th[p], N)
            assert abs(st["hh"][0] / hh - 1) < 1e-12
            assert abs(st["dh"][0] - dh) < 1e-11 * abs(dh) + 1e-12 * math.sqrt(hh)
        st1 = _stats(ds, th[p], 1)
        assert abs(st1["ups"][0] / (abs(dh) ** 2 / hh) - 1) < 1e-11


def test_semicoherent_overlap_inequalities():
    """Cauchy-Schwarz: hat O_N^2 <= <h|h> Upsilon_N, with equality at N = 1;
    per-segment phase maximisation: log hat L_N >= max_phi log L, equal at
    N = 1; splitting segments (nested explicit edges) cannot lower hat O_N
    (triangle inequality, eq:semi-coherent_O)."""
    ds = D.lisa_small(seed=13)
    th = D.lisa_particles(8, seed=42)
    th[0] = ds.injection
    dd = O.data_norm(ds.grid, ds.d_ri, ds.psd)
    for N in (1, 4, 32):
        st = _stats(ds, th, N, G=16)
        ok = np.isfinite(st["ups"]) & (st["hh"] > 0)
        lhs, rhs = st["overlap"][ok] ** 2, st["hh"][ok] * st["ups"][ok]
        if N == 1:
            assert np.allclose(lhs, rhs, rtol=1e-12, atol=0)
        else:
            assert np.all(lhs <= rhs * (1 + 1e-12))
        amp = 0.7 * st["overlap"][ok] / st["hh"][ok]
        semi, coh = O.loglike(dd, {k: v[ok] for k, v in st.items()}, amp)
        if N == 1:
            assert np.allclose(semi, coh, rtol=0, atol=1e-9 * dd)
        else:
            assert np.all(semi >= coh - 1e-9 * dd)
    K = ds.grid.K
    coarse = np.linspace(0, K, 5).astype(np.int64)
    fine = np.linspace(0, K, 17).astype(np.int64)
    assert set(coarse) <= set(fine)
    oc = _stats(ds, th, 4, O.SEG_EXPLICIT, edges=coarse)["overlap"]
    of = _stats(ds, th, 16, O.SEG_EXPLICIT, edges=fine)["overlap"]
    ok = np.isfinite(oc)
    assert np.all(of[ok] >= oc[ok] * (1 - 1e-13))


# ---------------------------------------------------------------- noise realisations (Sec 5.1)
def test_noise_counter_layout_and_box_muller():
    """One element by hand: the Philox4x32-10 block of counter (k, channel, r,
    'nois') and key (seed low, seed high) gives two 52-bit uniforms, and
    Box-Muller turns them into the element's real and imaginary parts."""
    ds = D.lisa_small(noise=False)
    seed, r = 0x1234_5678_9ABC, 7
    n = O.noise(ds.grid, ds.psd, seed, r)
    for a, k in ((0, 0), (1, 12345), (0, ds.grid.K - 1)):
        o = O.philox4x32_10([k, a, r, 0x6E6F6973], [seed & 0xFFFFFFFF, seed >> 32])
        u1 = (((o[0] >> 6) << 26 | (o[1] >> 6)) + 0.5) * 2.0 ** -52
        u2 = (((o[2] >> 6) << 26 | (o[3] >> 6)) + 0.5) * 2.0 ** -52
        rad = math.sqrt(-2.0 * math.log(u1))
        sig = math.sqrt(ds.psd[a, k] / (4.0 * ds.grid.df))
        assert abs(n[a, k] - sig * rad * complex(math.cos(2 * math.pi * u2), math.sin(2 * math.pi * u2))) <= 1e-15 * sig * rad


def test_noise_is_gaussian_with_the_inner_product_variance():
    """Whitened samples are standard normal (KS), and over realisations
    <n|h> has mean 0 and variance <h|h> (eqn:inner_prod convention)."""
    from scipy import stats

    ds = D.lisa_small(noise=False, snr=17.0)
    z = O.noise(ds.grid, ds.psd, 99, 0) / np.sqrt(ds.psd / (4.0 * ds.grid.df))
    assert stats.kstest(z.real.ravel(), "norm").pvalue > 1e-3
    assert stats.kstest(z.imag.ravel(), "norm").pvalue > 1e-3
    assert abs(np.corrcoef(z.real.ravel(), z.imag.ravel())[0, 1]) < 0.03
    h = ds.d
    hh = D.inner(ds.grid, ds.psd, h, h)
    x = np.array([D.inner(ds.grid, ds.psd, O.noise(ds.grid, ds.psd, 99, r), h) for r in range(400)])
    assert abs(x.mean()) < 4 * math.sqrt(hh / len(x))
    # sample variance of 400 normals: relative sd sqrt(2/399) ~ 0.071
    assert abs(x.var(ddof=1) / hh - 1) < 4 * math.sqrt(2 / 399)
