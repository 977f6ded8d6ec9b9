"""Parity of the full frequency-domain response (Sec 4 response paragraph:
TDI A/E (and T) transfer functions with finite arm length) through the C ABI against
the oracle: the template per bin, supports and equal-[h|h] edges, Upsilon_N
in FP64 and mixed precision, per-segment sums, the likelihood statistics and
a noise-free injection.

Tolerances as for the low-frequency response: template within 1e-10 of
max|h| (phase Taylor remainder 1e-12 cycles, response interpolation 1e-11),
Upsilon_N within 1e-9 (FP64) and 1e-5 (mixed) floored relative error
(floor 2 N_eff), edges bit-exact except at a rounding tie of the oracle's
cumulative, where the row is compared with the oracle on the GPU's edges
(tests/parity.py).
"""
import numpy as np
import pytest

import oracle as O
import synth
from tests import datasets as D
from tests import parity as PT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_13170_amd import B  # noqa: E402


def _ctx(ds, N, mode=B.SCS_SEG_EQUAL_SNR, G=1):
    g = ds.grid
    h = B.scs_ctx_create(0)
    B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
    m = ds.model
    B.scs_set_model(h, m.pn_order, m.response, m.support, m.t_obs)
    B.scs_define_segmentation(h, N, mode, G)
    return h


@pytest.mark.parametrize("n_chan", [2, 3])
def test_template_matches_oracle(n_chan):
    ds = D.lisa_small(noise=False, response=O.RESP_LISA_FD, n_chan=n_chan)
    h = _ctx(ds, 1)
    try:
        ths = [ds.injection] + list(D.lisa_particles(4, seed=78))
        for th in ths:
            out = torch.empty((n_chan, ds.grid.K, 2), dtype=torch.float64, device="cuda")
            B.scs_waveform(h, torch.tensor(np.ascontiguousarray(th), device="cuda"), out)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            gc = got[..., 0] + 1j * got[..., 1]
            ref = O.template(ds.grid, ds.model, th)
            nz = np.abs(ref) > 0
            assert np.array_equal(nz, np.abs(gc) > 0), "supports differ"
            err = np.abs(gc - ref)[nz].max() / np.abs(ref).max()
            # the full response differs from the low-frequency one by O(1) here
            g2 = O.Grid(ds.grid.K, ds.grid.k0, ds.grid.df, 2)
            lf = O.template(g2, O.Model(pn_order=ds.model.pn_order, response=O.RESP_LISA_LF_AE,
                                        support=ds.model.support, t_obs=ds.model.t_obs), th)
            dif = np.abs(lf - ref[:2])[nz[:2]].max() / np.abs(ref).max()
            print(f"full-response template max err / max|h| {err:.3g} (LF differs by {dif:.3g})")
            assert err < 1e-10 and dif > 0.1
    finally:
        B.scs_ctx_destroy(h)


@pytest.mark.parametrize("N,mode,G,n_chan", [(1, B.SCS_SEG_EQUAL_SNR, 1, 2), (8, B.SCS_SEG_EQUAL_SNR, 16, 2),
                                             (64, B.SCS_SEG_EQUAL_SNR, 1, 2), (37, B.SCS_SEG_UNIFORM, 1, 2),
                                             (1, B.SCS_SEG_EQUAL_SNR, 1, 3), (16, B.SCS_SEG_EQUAL_SNR, 16, 3),
                                             (64, B.SCS_SEG_EQUAL_SNR, 1, 3)])
def test_upsilon_matches_oracle(N, mode, G, n_chan):
    ds = D.lisa_small(seed=41, response=O.RESP_LISA_FD, n_chan=n_chan)
    th = D.lisa_particles(40, seed=42)
    th[:4] = synth.near_injection(ds.injection, 4, seed=43)
    th[4, 0] = -1.0      # invalid: NaN
    th[5, 2] = 0.0195    # empty support: 0
    ref = O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, th, N, mode, G, want_seg=True, want_bounds=True)
    h = _ctx(ds, N, mode, G)
    try:
        tht = torch.tensor(np.ascontiguousarray(th), device="cuda")
        u = torch.empty(th.shape[0], dtype=torch.float64, device="cuda")
        seg = torch.empty((th.shape[0], N, 3), dtype=torch.float64, device="cuda")
        B.scs_evaluate(h, tht, u, B.SCS_PREC_FP64, seg)
        torch.cuda.synchronize()
        got, sg = u.cpu().numpy(), seg.cpu().numpy()
        assert np.isnan(got[4]) and got[5] == 0.0
        sup, bnd = B.scs_last_bounds(h, th.shape[0], N)
        ok = np.isfinite(ref["ups"])
        assert np.array_equal(sup[ok], ref["support"][ok])
        PT.check_rows(ds, th, got, ref, bnd, G, PT.TOL64, mode, what=f"{n_chan} channels, N={N} fp64")
        same = ok & np.all(bnd == ref["bounds"], axis=1)
        rs = ref["seg"][same]
        live = rs[..., 2] > 0
        herr = np.abs(sg[same][..., 2][live] / rs[..., 2][live] - 1).max()
        print(f"{n_chan} channels, N={N}: H max rel err {herr:.3g} on {same.sum()} rows with the oracle's edges")
        assert herr < 5e-11
        B.scs_evaluate(h, tht, u, B.SCS_PREC_MIXED)
        torch.cuda.synchronize()
        PT.check_rows(ds, th, u.cpu().numpy(), ref, bnd, G, PT.TOLMIX, mode, what=f"N={N} mixed")
    finally:
        B.scs_ctx_destroy(h)


@pytest.mark.parametrize("n_chan", [2, 3])
def test_noise_free_injection_and_statistics(n_chan):
    """d = A h(theta*): Upsilon_N = rho^2 for every N, log L = 0 at the true
    amplitude, and the statistics rows against the oracle's."""
    ds = D.lisa_small(noise=False, snr=17.0, response=O.RESP_LISA_FD, n_chan=n_chan)
    for N in (1, 16):
        h = _ctx(ds, N, G=16)
        try:
            th = np.ascontiguousarray(ds.injection[None, :])
            st = np.empty((1, B.SCS_NSTATS))
            B.scs_evaluate_stats(h, th, st)
            print(f"N={N}: Upsilon at the injection {st[0, 0]:.12f} (rho^2 = {ds.snr ** 2})")
            assert abs(st[0, 0] / ds.snr ** 2 - 1) < 1e-9
            ref = O.likelihood_stats(ds.grid, ds.model, ds.d_ri, ds.psd, th, N, O.SEG_EQUAL_SNR, 16)
            assert abs(st[0, 2] / ref["hh"][0] - 1) < 5e-11
            dd = B.scs_data_norm(h)
            amp = np.array([ds.snr / np.sqrt(st[0, 2])])
            semi, coh = np.empty(1), np.empty(1)
            B.scs_loglike(h, st, amp, np.zeros(1), semi, coh)
            assert abs(semi[0]) < 1e-9 * dd and abs(coh[0]) < 1e-9 * dd
        finally:
            B.scs_ctx_destroy(h)


@pytest.mark.parametrize("n_chan", [2, 3])
def test_full_response_lisa1m_full_size_sampled(n_chan):
    """The benchmark's full-response configurations at their full size (2^20
    bins, 10^4 particles, N = 1024, G = 1024, the TDI noise PSDs) in the launch
    configurations `bench.py --response fd` (A, E) and `--response fd3`
    (A, E, T) time; the oracle recomputes a seeded sample of particles one by
    one."""
    w = synth.workload("lisa1m")
    g = O.Grid(w.grid.K, w.grid.k0, w.grid.df, n_chan)
    m = O.Model(pn_order=7, response=O.RESP_LISA_FD, support=O.SUPPORT_TOBS, t_obs=w.grid.t_obs)
    psd = synth.lisa_tdi_psd(w.grid.freqs())[:n_chan]
    ds = D.make(g, m, psd, w.injection, w.snr, w.seed, True, w.prior_lo, w.prior_hi)
    theta = synth.workload_particles(w)
    theta[:2] = synth.near_injection(w.injection, 2, seed=6, lo=w.prior_lo, hi=w.prior_hi)
    N = w.N
    h = _ctx(ds, N, B.SCS_SEG_EQUAL_SNR, w.G)
    try:
        tht = torch.tensor(theta, device="cuda")
        u = torch.empty(theta.shape[0], dtype=torch.float64, device="cuda")
        B.scs_evaluate(h, tht, u)
        torch.cuda.synchronize()
        got = u.cpu().numpy()
        sup, bnd = B.scs_last_bounds(h, theta.shape[0], N)
        B.scs_evaluate(h, tht, u, B.SCS_PREC_MIXED)
        torch.cuda.synchronize()
        gm = u.cpu().numpy()
        assert np.all(np.isfinite(got)) and np.all(got >= 0)
        idx = np.concatenate([[0, 1], np.random.default_rng(4).choice(np.arange(2, len(theta)), 4, replace=False)])
        ref = O.evaluate(g, m, ds.d_ri, psd, theta[idx], N, O.SEG_EQUAL_SNR, w.G, want_bounds=True)
        assert np.array_equal(sup[idx], ref["support"])
        PT.check_rows(ds, theta[idx], got[idx], ref, bnd[idx], w.G, PT.TOL64,
                      what=f"full response, {n_chan} channels, 2^20 bins, sampled fp64")
        PT.check_rows(ds, theta[idx], gm[idx], ref, bnd[idx], w.G, PT.TOLMIX,
                      what=f"full response, {n_chan} channels, 2^20 bins, sampled mixed")
        print(f"Upsilon near the injection {got[:2]} (oracle {ref['ups'][:2]})")
    finally:
        B.scs_ctx_destroy(h)
