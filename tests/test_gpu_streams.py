"""One theta against many data streams (Sec 5.1): the device's noise
realisations against the oracle's own Philox / Box-Muller generator, the
streamed statistics against the oracle on each realisation, and at scale the
sampling law Upsilon_N ~ chi^2_{2N}(rho^2) that holds at fixed theta
(eqn:CLTdist_noise, eqn:CLTdist_signal give its moments).

Tolerances: realisations within 1e-13 of sqrt(S / 4df) + |d| per element
(the two sides' log and sin / cos may differ in the last bit); statistics as
in the likelihood tests (1e-9 floored relative on Upsilon_N, 1e-9 on the
Cauchy-Schwarz scale for hat O_N and <d|h>, 5e-11 relative on <h|h>).
"""
import math

import numpy as np
import pytest

import oracle as O
import synth
from tests import datasets as D
from tests import parity as PT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_13170_amd import B  # noqa: E402


def _ctx(ds, N, G=1):
    g = ds.grid
    h = B.scs_ctx_create(0)
    B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
    m = ds.model
    B.scs_set_model(h, m.pn_order, m.response, m.support, m.t_obs)
    B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, G)
    return h


def test_realisations_and_streamed_statistics_match_oracle():
    ds = D.lisa_small(seed=25)
    g = ds.grid
    seed, r0, R, scale = 0xC0FFEE_1234, 3, 5, 0.5
    th = np.stack([ds.injection, D.lisa_particles(1, seed=250)[0]])
    h = _ctx(ds, 8)
    try:
        streams = torch.empty((g.n_chan, g.K, R, 2), dtype=torch.float64, device="cuda")
        B.scs_make_realisations(h, streams, seed, r0, scale)
        torch.cuda.synchronize()
        got = streams.cpu().numpy()
        datas = []
        sig = np.sqrt(ds.psd / (4.0 * g.df))
        for r in range(R):
            want = scale * ds.d + O.noise(g, ds.psd, seed, r0 + r)
            gr = got[:, :, r, 0] + 1j * got[:, :, r, 1]
            assert np.max(np.abs(gr - want) / (sig + np.abs(scale * ds.d))) < 1e-13
            datas.append(np.stack([want.real, want.imag], -1))
        stats = torch.empty((R, B.SCS_NSTATS), dtype=torch.float64, device="cuda")
        for N in (1, 8):
            B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, 1)
            for p in range(th.shape[0]):
                B.scs_evaluate_streams(h, th[p], streams, stats)
                s = stats.cpu().numpy()
                # the edges depend on theta only: N_eff from the oracle's
                neff = PT.n_eff(O.evaluate(g, ds.model, datas[0], ds.psd, th[p:p + 1], N, O.SEG_EQUAL_SNR, 1,
                                           want_bounds=True)["bounds"])
                for r in range(R):
                    ref = O.likelihood_stats(g, ds.model, datas[r], ds.psd, th[p:p + 1], N, O.SEG_EQUAL_SNR, 1)
                    dd = O.data_norm(g, datas[r], ds.psd)
                    e_ups = float(PT.floored(s[r:r + 1, 0], ref["ups"], neff)[0])
                    cs = math.sqrt(dd * ref["hh"][0])
                    e_ov = abs(s[r, 1] - ref["overlap"][0]) / cs
                    e_dh = abs(complex(s[r, 3], s[r, 4]) - ref["dh"][0]) / cs
                    e_hh = abs(s[r, 2] / ref["hh"][0] - 1)
                    assert e_ups < 1e-9 and e_ov < 1e-9 and e_dh < 1e-9 and e_hh < 5e-11, (N, p, r, e_ups, e_ov,
                                                                                            e_dh, e_hh)
                print(f"N={N} particle {p}: streamed statistics match the oracle on {R} realisations")
        # an invalid theta gives NaN rows
        bad = ds.injection.copy()
        bad[0] = -1.0
        B.scs_evaluate_streams(h, bad, streams, stats)
        assert np.all(np.isnan(stats.cpu().numpy()))
    finally:
        B.scs_ctx_destroy(h)


@pytest.mark.parametrize("snr", [0.0, 17.0])
def test_chi2_law_at_scale(snr):
    """4000 realisations at the true theta: with noise only Upsilon_N ~ chi^2_{2N},
    with the signal chi^2_{2N}(rho^2) (each segment is a non-central chi^2 with
    two degrees of freedom at fixed theta and edges)."""
    from scipy import stats as S

    ds = D.lisa_small(noise=False, snr=17.0)
    g = ds.grid
    R = 4000
    h = _ctx(ds, 1)
    try:
        streams = torch.empty((g.n_chan, g.K, R, 2), dtype=torch.float64, device="cuda")
        B.scs_make_realisations(h, streams, 20240813, 0, 1.0 if snr > 0 else 0.0)
        st = torch.empty((R, B.SCS_NSTATS), dtype=torch.float64, device="cuda")
        for N in (1, 8, 32):
            B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, 1)
            B.scs_evaluate_streams(h, ds.injection, streams, st)
            u = st[:, 0].cpu().numpy()
            law = S.ncx2(2 * N, snr ** 2) if snr > 0 else S.chi2(2 * N)
            p = S.kstest(u, law.cdf).pvalue
            mean, var = 2 * N + snr ** 2, 4 * N + 4 * snr ** 2
            print(f"snr {snr} N={N}: mean {u.mean():.3f} (law {mean}), var {u.var():.2f} (law {var}), KS p {p:.3g}")
            assert p > 1e-3
            assert abs(u.mean() - mean) < 4 * math.sqrt(var / R)
    finally:
        B.scs_ctx_destroy(h)


def test_streams_lisa1m_full_size_sampled():
    """The configuration `bench.py --mode streams` times, at its full grid: the
    GW150914-like injection alone in the 2^20-bin A+E band at SNR 20 (G =
    1024), realisations generated on the device, then the streamed statistics
    of the injected theta at N in {1, 10, 50, 100}; three realisations
    recomputed by the oracle (its own noise generator and statistics).  The
    benchmark streams 1024 realisations; 64 here keep the test's memory small,
    and the per-realisation work is the same."""
    w = synth.workload("lisa1m")
    g = O.Grid(w.grid.K, w.grid.k0, w.grid.df, 2)
    m = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=w.grid.t_obs)
    psd = synth.psd_arrays(w)
    ds = D.make(g, m, psd, w.injection, 20.0, w.seed, False)
    seed, R = synth.BASE_SEED + 51, 64
    h = B.scs_ctx_create(0)
    try:
        B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(psd), g.k0 * g.df, g.df)
        B.scs_set_model(h, 7, m.response, m.support, m.t_obs)
        B.scs_define_segmentation(h, 1, B.SCS_SEG_EQUAL_SNR, w.G)
        streams = torch.empty((2, g.K, R, 2), dtype=torch.float64, device="cuda")
        B.scs_make_realisations(h, streams, seed, 0, 1.0)
        stats = torch.empty((R, B.SCS_NSTATS), dtype=torch.float64, device="cuda")
        sample = [0, 17, 63]
        datas = {}
        for r in sample:
            n = ds.d + O.noise(g, psd, seed, r)
            datas[r] = np.stack([n.real, n.imag], -1)
        worst = 0.0
        for N in (1, 10, 50, 100):
            B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, w.G)
            B.scs_evaluate_streams(h, w.injection, streams, stats)
            s = stats.cpu().numpy()
            assert np.all(np.isfinite(s[:, 0]))
            neff = PT.n_eff(O.evaluate(g, m, datas[sample[0]], psd, w.injection[None, :], N, O.SEG_EQUAL_SNR, w.G,
                                       want_bounds=True)["bounds"])
            for r in sample:
                ref = O.likelihood_stats(g, m, datas[r], psd, w.injection[None, :], N, O.SEG_EQUAL_SNR, w.G)
                e = float(PT.floored(s[r:r + 1, 0], ref["ups"], neff)[0])
                worst = max(worst, e)
                assert e < 1e-9 and abs(s[r, 2] / ref["hh"][0] - 1) < 5e-11, (N, r, e)
        print(f"streams, 2^20 bins: sampled realisations, max floored rel err {worst:.3g}")
    finally:
        B.scs_ctx_destroy(h)
