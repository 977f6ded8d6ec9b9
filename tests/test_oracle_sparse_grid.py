"""What the paper's sparse-grid evaluation (Sec 4: waveform and response on a
grid coarser than the FFT grid by 1000, cubic-spline interpolated onto it)
would cost in accuracy, measured with the oracle on the 2^20-bin workload:
the interpolated phase against the exact one at every in-support bin, and
the overlap lost at the injection.  The library evaluates the phase per
block with a remainder bound of 1e-12 cycles instead (no interpolation)."""
import math

import numpy as np
import pytest

import oracle as O
import synth

interpolate = pytest.importorskip("scipy.interpolate")


def test_cubic_spline_on_a_grid_coarser_by_1000():
    w = synth.workload("lisa1m")
    g = w.grid
    m = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=g.t_obs)
    f = (g.k0 + np.arange(g.K)) * g.df
    frac, whole, t, _ = O.phase(m, w.injection, f)
    k = np.flatnonzero((f >= w.injection[2]) & (t < g.t_obs))
    # the phase relative to its value at the first support bin, so that the
    # differences keep their precision in double
    ph = (whole[k] - whole[k[0]]) + (frac[k] - frac[k[0]])
    nodes = np.append(np.arange(0, k.size, 1000), k.size - 1)
    sp = interpolate.CubicSpline(f[k][nodes], ph[nodes])
    err = sp(f[k]) - ph
    emax = np.abs(err).max()
    print(f"{k.size} bins, {nodes.size} nodes: spline phase error max {emax:.3g} cycles, "
          f"median {np.median(np.abs(err)):.3g}")
    # about 1e-6 cycles: far above the 1e-12-cycle bound of the block polynomials ...
    assert 1e-8 < emax < 1e-4
    # ... yet second order in Upsilon: the overlap of e^{2 pi i err} with 1
    loss = 1.0 - abs(np.mean(np.exp(2j * math.pi * err)))
    print(f"overlap lost at the injection: {loss:.3g}")
    assert loss < 1e-9


# ---------------------------------------------------------------- the sparse-grid mode of the oracle
# (Sec 4: waveform and response on a coarse grid, cubic-spline interpolated
# onto the FFT grid).  Pinned against scipy's not-a-knot cubic spline through
# node values computed independently from the oracle's exact phase, time and
# antenna patterns, and against the exact template at the nodes.

def _sparse_model(base, stride):
    return O.Model(pn_order=base.pn_order, response=base.response, support=base.support, t_obs=base.t_obs,
                   sparse_stride=stride)


def _nodes(klo, khi, S):
    x = [klo] + list(range((klo // S + 1) * S, khi - 1, S))
    if khi - 1 > klo:
        x.append(khi - 1)
    return np.array(x)


def _scipy_spline_template(ds, theta, S):
    """The sparse-grid template rebuilt with scipy: node quantities (phase in
    cycles with the Doppler term, the A and E responses) from the oracle's
    exact phase, SPA time and antenna patterns; scipy's not-a-knot cubic
    spline of each onto every support bin; h = f^-7/6 R e^{-2 pi i phase}."""
    g, m = ds.grid, ds.model
    f = g.freqs
    frac, whole, t, _ = O.phase(m, theta, f)
    # the support as the oracle decides it (its f_low comparison is exact)
    klo, khi = (int(v) for v in O.evaluate(g, m, ds.d_ri, ds.psd, theta[None, :], 1)["support"][0])
    x = _nodes(klo, khi, S)
    ph0 = frac[klo]  # the integer part of the phase is no phase
    q = []
    for kk in x:
        F, dop, _ = O.response(m, theta, t[kk])
        ph = (whole[kk] - whole[klo]) + (frac[kk] - frac[klo]) + dop * f[kk]
        ap, ax = 0.5 * (1 + math.cos(theta[5]) ** 2), math.cos(theta[5])
        q.append([ph, F[0, 0] * ap, -F[0, 1] * ax, F[1, 0] * ap, -F[1, 1] * ax])
    q = np.array(q)
    kk = np.arange(klo, khi)
    vals = [interpolate.CubicSpline(x, q[:, c], bc_type="not-a-knot")(kk) if len(x) > 2 else
            np.interp(kk, x, q[:, c]) for c in range(5)]
    tot = vals[0] + ph0
    amp = f[kk] ** (-7.0 / 6.0)
    e = np.exp(-2j * math.pi * np.mod(tot, 1.0))
    h = np.zeros((2, g.K), dtype=complex)
    for a in range(2):
        h[a, kk] = amp * (vals[1 + 2 * a] + 1j * vals[2 + 2 * a]) * e
    return h, x


@pytest.mark.parametrize("S", [128, 1024])
def test_sparse_template_is_the_not_a_knot_spline(S):
    from tests import datasets as D

    ds = D.lisa_small(seed=91, noise=False)
    ms = _sparse_model(ds.model, S)
    for th in [ds.injection] + list(D.lisa_particles(3, seed=92)):
        got = O.template(ds.grid, ms, th)
        want, x = _scipy_spline_template(ds, th, S)
        scale = np.abs(want).max()
        err = np.abs(got - want).max() / scale
        exact = O.template(ds.grid, ds.model, th)
        at_nodes = np.abs(got[:, x] - exact[:, x]).max() / scale
        between = np.abs(got - exact).max() / scale
        print(f"S = {S}, {len(x)} nodes: spline vs scipy {err:.3g}, at nodes vs exact {at_nodes:.3g}, "
              f"between nodes vs exact {between:.3g}")
        # the same spline to scipy's float64 arithmetic (other end conditions,
        # natural or clamped, differ by orders of magnitude more near the ends)
        assert err < 1e-9
        # a spline passes through its nodes: the node phases are quad precision,
        # the per-bin template's extended precision (~1e-13 cycles at ~1e6)
        assert at_nodes < 5e-12
        assert between > 1e3 * at_nodes or S == 128  # interpolation, not evaluation


def test_sparse_statistic_against_brute_force():
    """Upsilon_N with the sparse-grid template: the oracle's evaluate against
    the statistic summed here from the scipy-built template over the
    oracle's (exact-weight) edges; and at the injection, noise-free, the
    overlap lost to interpolation is second order (Upsilon_N within 1e-6 of
    rho^2)."""
    from tests import datasets as D

    ds = D.lisa_small(seed=93)
    S, N = 512, 8
    ms = _sparse_model(ds.model, S)
    th = D.lisa_particles(3, seed=94)
    th[0] = ds.injection
    r = O.evaluate(ds.grid, ms, ds.d_ri, ds.psd, th, N, O.SEG_EQUAL_SNR, 16, want_bounds=True)
    r_exact = O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, th, N, O.SEG_EQUAL_SNR, 16, want_bounds=True)
    assert np.array_equal(r["bounds"], r_exact["bounds"])  # edges keep the exact weights
    for p in range(th.shape[0]):
        h, _ = _scipy_spline_template(ds, th[p], S)
        b = r["bounds"][p]
        ups = 0.0
        for n in range(N):
            sl = slice(b[n], b[n + 1])
            Z = np.sum(ds.d[:, sl] * np.conj(h[:, sl]) / ds.psd[:, sl])
            H = np.sum(np.abs(h[:, sl]) ** 2 / ds.psd[:, sl])
            if H > 0:
                ups += 4 * ds.grid.df * abs(Z) ** 2 / H
        assert abs(r["ups"][p] - ups) <= 1e-8 * max(ups, 2 * N), (p, r["ups"][p], ups)
    clean = D.lisa_small(seed=93, noise=False)
    u = O.evaluate(clean.grid, ms, clean.d_ri, clean.psd, clean.injection[None, :], N, O.SEG_EQUAL_SNR, 16)["ups"][0]
    print(f"noise-free injection, sparse template: Upsilon_{N} = {u:.9f} (rho^2 = {clean.snr ** 2})")
    assert 0 < clean.snr ** 2 - u < 1e-6 * clean.snr ** 2


def test_sparse_small_supports():
    """Supports of one, two and three nodes: the constant, the line and the
    parabola (scipy's not-a-knot with three points) through them."""
    from tests import datasets as D

    ds = D.lisa_small(seed=95, noise=False)
    th = ds.injection.copy()
    cases = [(0.018999, 4096, 1e7, 2), (0.01895, 512, 1e7, 3), (0.0185, 1024, 1.0, 1)]
    for fl, S, t_obs, n_nodes in cases:
        th[2] = fl
        dsm = D.Dataset(ds.grid, O.Model(pn_order=ds.model.pn_order, response=ds.model.response,
                                         support=ds.model.support, t_obs=t_obs), ds.psd, ds.d, th, 0.0, None, None)
        got = O.template(dsm.grid, _sparse_model(dsm.model, S), th)
        want, x = _scipy_spline_template(dsm, th, S)
        nz = np.abs(want) > 0
        print(f"f_low {fl}, stride {S}: {len(x)} nodes, {nz[0].sum()} bins")
        assert len(x) == n_nodes
        assert np.array_equal(np.abs(got) > 0, nz)
        assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()


def test_sparse_phase_spline_precision_at_a_one_bin_end_interval():
    """Rounding of the node phases, multiplied by a short end interval.  With
    nodes every S bins and a support that ends one bin after the last
    multiple of S, the not-a-knot condition ties the last two intervals, and
    an error e in a node phase moves the spline next to it by ~0.75 S e.  The
    phase spline here is rebuilt in 40-digit arithmetic (node phases from the
    2PN series, the not-a-knot system solved densely by mpmath), and the
    oracle's sparse-grid template must carry the same interpolation error
    (spline minus exact phase) at every bin to 5e-12 cycles; node phases
    rounded at ~2e-13 cycles (extended precision at ~4e6 cycles) would miss it
    by more than an order of magnitude next to the short interval."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    S = 1024
    K = 4 * S + 2  # nodes 0, S, 2S, 3S, 4S and K - 1 = 4S + 1: the last interval is one bin
    # the 2^20-bin grid's bin width, from 0.018 Hz (where the interpolation
    # error of the phase is ~1e-7 cycles, so that its difference is a phase)
    spec = synth.GridSpec(1 << 20)
    k0 = int(round(0.018 / spec.df))
    grid = O.Grid(K, k0, spec.df, 1)
    t_obs = 1.0 / spec.df
    model = O.Model(pn_order=4, response=O.RESP_NONE, support=O.SUPPORT_FULL, t_obs=t_obs, sparse_stride=S)
    th = np.array([28.0, float(synth.eta_from_q(0.8)), k0 * spec.df, 0, 0, 0, 0])
    eta, mc = mp.mpf(th[1]), mp.mpf(th[0])
    tsun = mp.mpf("1.32712440018e20") / mp.mpf(299792458) ** 3
    piM = mp.pi * mc * eta ** mp.mpf("-0.6") * tsun
    pref = 3 / (256 * mp.pi * eta)
    psi2 = mp.mpf(3715) / 756 + 55 * eta / 9
    psi3 = -16 * mp.pi
    psi4 = mp.mpf(15293365) / 508032 + 27145 * eta / 504 + 3085 * eta ** 2 / 72

    def series(v):
        return (1 + psi2 * v ** 2 + psi3 * v ** 3 + psi4 * v ** 4) / v ** 5

    def dseries(v):  # f d/df of the series, dv/df = v / (3 f)
        return (-5 + -3 * psi2 * v ** 2 - 2 * psi3 * v ** 3 - psi4 * v ** 4) / v ** 5 / 3

    fl = mp.mpf(k0) * mp.mpf(spec.df)
    tc = -pref * dseries(mp.cbrt(piM * fl)) / fl

    def phase(k):
        f = mp.mpf(int(k0 + k)) * mp.mpf(spec.df)
        return f * tc - mp.mpf(1) / 8 + pref * series(mp.cbrt(piM * f))

    x = _nodes(0, K, S)
    assert list(x) == [0, S, 2 * S, 3 * S, 4 * S, K - 1]
    y = [phase(int(k)) for k in x]
    n = len(x) - 1
    h = [mp.mpf(int(x[j + 1] - x[j])) for j in range(n)]
    # unknowns M_0 .. M_n: n - 1 continuity rows and two not-a-knot rows
    A = mp.zeros(n + 1, n + 1)
    r = mp.zeros(n + 1, 1)
    for i in range(1, n):
        A[i, i - 1], A[i, i], A[i, i + 1] = h[i - 1], 2 * (h[i - 1] + h[i]), h[i]
        r[i] = 6 * ((y[i + 1] - y[i]) / h[i] - (y[i] - y[i - 1]) / h[i - 1])
    A[0, 0], A[0, 1], A[0, 2] = -1 / h[0], 1 / h[0] + 1 / h[1], -1 / h[1]
    A[n, n - 2], A[n, n - 1], A[n, n] = -1 / h[n - 2], 1 / h[n - 2] + 1 / h[n - 1], -1 / h[n - 1]
    M = mp.lu_solve(A, r)
    # compared: the interpolation error (spline minus exact phase) of the
    # oracle and of the 40-digit rebuild, so that the oracle's own t_c (a
    # phase linear in f, which any spline reproduces) drops out
    sp = O.template(grid, model, th)[0]
    ex = O.template(grid, O.Model(pn_order=4, response=O.RESP_NONE, support=O.SUPPORT_FULL, t_obs=t_obs), th)[0]
    got = np.angle(sp / ex) / (2 * math.pi)  # spline minus exact phase, cycles (the template is e^{-2 pi i phase})
    got = -got
    worst = 0.0
    for k in range(K):
        j = min(int(np.searchsorted(x, k, side="right")) - 1, n - 1)
        u, hj = mp.mpf(int(k - x[j])), h[j]
        b = (y[j + 1] - y[j]) / hj - hj * (2 * M[j] + M[j + 1]) / 6
        q = y[j] + u * (b + u * (M[j] / 2 + u * (M[j + 1] - M[j]) / (6 * hj)))
        worst = max(worst, abs(float(q - phase(k)) - got[k]))
    print(f"one-bin end interval, S = {S}: interpolation error of the sparse-grid phase against the 40-digit "
          f"spline's, max difference {worst:.3g} cycles")
    assert worst < 5e-12
