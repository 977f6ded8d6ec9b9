"""Likelihood epilogues (Sec 2.1 - 2.2) on the GPU against the oracle: the
per-particle statistics (Upsilon_N, hat O_N, <h|h>, <d|h>) of the
generate-and-reduce, <d|d> of the loaded data, and the semi-coherent and
coherent log-likelihoods.

Tolerances: Upsilon_N as the parity tests (1e-9 floored relative in FP64,
1e-5 mixed).  hat O_N and <d|h> are compared on the Cauchy-Schwarz scale
sqrt(<d|d> <h|h>) that bounds them; <h|h> relative, where the response
interpolation budget (1e-11 on R, 2e-11 on |R|^2) is the floor.  The
log-likelihoods on the scale <d|d> + A^2 <h|h> of their terms.
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


def _ctx(ds, N, G=1):
    g = ds.grid
    h = B.scs_ctx_create(0)
    B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
    m = ds.model
    B.scs_set_model(h, m.pn_order, m.response, m.support, m.t_obs)
    B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, G)
    return h


def _check(st, ref, dd, N, tol_ups, tol_lin, tol_hh):
    ok = np.isfinite(ref["ups"])
    assert np.all(np.isnan(st[~ok]))
    s, r = st[ok], {k: v[ok] for k, v in ref.items()}
    e_ups = PT.floored(s[:, 0], r["ups"], PT.n_eff(r["bounds"]))
    scale = np.sqrt(dd * np.maximum(r["hh"], 1e-300))
    e_ov = np.abs(s[:, 1] - r["overlap"]) / scale
    e_dh = np.abs((s[:, 3] + 1j * s[:, 4]) - r["dh"]) / scale
    live = r["hh"] > 0
    e_hh = np.abs(s[live, 2] / r["hh"][live] - 1)
    print(f"N={N}: ups {e_ups.max():.3g} overlap {e_ov.max():.3g} dh {e_dh.max():.3g} hh {e_hh.max():.3g}")
    assert e_ups.max() < tol_ups and e_ov.max() < tol_lin and e_dh.max() < tol_lin and e_hh.max() < tol_hh
    assert np.all(s[~live] == 0.0)


def test_statistics_and_loglike_match_oracle():
    ds = D.lisa_small(seed=23)
    th = D.lisa_particles(48, seed=230)
    th[0] = ds.injection
    th[1:5] = synth.near_injection(ds.injection, 4, seed=231)
    th[5, 0] = -1.0        # invalid: NaN row
    th[6, 2] = 0.0195      # empty support: zero row
    dd_ref = O.data_norm(ds.grid, ds.d_ri, ds.psd)
    for N in (1, 16, 64):
        h = _ctx(ds, N)
        try:
            dd = B.scs_data_norm(h)
            assert abs(dd / dd_ref - 1) < 1e-12
            ref = O.likelihood_stats(ds.grid, ds.model, ds.d_ri, ds.psd, th, N, O.SEG_EQUAL_SNR, 1)
            tht = torch.tensor(np.ascontiguousarray(th), device="cuda")
            st = torch.empty((th.shape[0], B.SCS_NSTATS), dtype=torch.float64, device="cuda")
            B.scs_evaluate_stats(h, tht, st)
            torch.cuda.synchronize()
            s64 = st.cpu().numpy()
            _check(s64, ref, dd, N, 1e-9, 1e-9, 5e-11)
            # Upsilon_N equals scs_evaluate's, bit for bit
            u = torch.empty(th.shape[0], dtype=torch.float64, device="cuda")
            B.scs_evaluate(h, tht, u)
            torch.cuda.synchronize()
            un = u.cpu().numpy()
            fin = np.isfinite(un)
            assert np.array_equal(un[fin], s64[fin, 0])
            # host pointers give the same rows
            sh = np.empty_like(s64)
            B.scs_evaluate_stats(h, np.ascontiguousarray(th), sh)
            assert np.array_equal(np.nan_to_num(sh), np.nan_to_num(s64))
            # mixed precision
            B.scs_evaluate_stats(h, tht, st, prec=B.SCS_PREC_MIXED)
            torch.cuda.synchronize()
            _check(st.cpu().numpy(), ref, dd, N, 1e-5, 1e-5, 1e-5)
            # log-likelihoods at seeded amplitudes and phases, on the device
            rng = np.random.default_rng(N)
            ok = np.isfinite(ref["ups"]) & (ref["hh"] > 0)
            amp = np.where(ok, rng.uniform(0.2, 1.5, th.shape[0]) * ref["overlap"] / np.where(ok, ref["hh"], 1.0), 1.0)
            phase = rng.uniform(-np.pi, np.pi, th.shape[0])
            st64 = torch.tensor(s64, device="cuda")
            semi = torch.empty(th.shape[0], dtype=torch.float64, device="cuda")
            coh = torch.empty_like(semi)
            cohmax = torch.empty_like(semi)
            ampt, pht = torch.tensor(amp, device="cuda"), torch.tensor(phase, device="cuda")
            B.scs_loglike(h, st64, ampt, pht, semi, coh)
            B.scs_loglike(h, st64, ampt, None, None, cohmax)
            torch.cuda.synchronize()
            rs, rc = O.loglike(dd_ref, ref, amp, phase)
            _, rcm = O.loglike(dd_ref, ref, amp)
            scale = dd_ref + amp ** 2 * np.where(ok, ref["hh"], 0.0)
            for got, want in ((semi, rs), (coh, rc), (cohmax, rcm)):
                e = np.abs(got.cpu().numpy()[ok] - want[ok]) / scale[ok]
                assert e.max() < 1e-9, e.max()
            # host arrays through the same kernel
            semi_h, coh_h = np.empty(th.shape[0]), np.empty(th.shape[0])
            B.scs_loglike(h, s64, amp, phase, semi_h, coh_h)
            assert np.array_equal(semi_h[ok], semi.cpu().numpy()[ok])
            assert np.array_equal(coh_h[ok], coh.cpu().numpy()[ok])
            # semi-coherent >= phase-maximised coherent, equal at N = 1
            sm, cm = semi.cpu().numpy()[ok], cohmax.cpu().numpy()[ok]
            if N == 1:
                assert np.allclose(sm, cm, rtol=0, atol=1e-9 * dd)
            else:
                assert np.all(sm >= cm - 1e-9 * dd)
        finally:
            B.scs_ctx_destroy(h)


def test_noise_free_injection_loglike_zero():
    """d = A h(theta*): at the true amplitude and zero phase both
    log-likelihoods vanish (to the scale of their terms)."""
    ds = D.lisa_small(noise=False, snr=17.0)
    for N in (1, 32):
        h = _ctx(ds, N, G=16)
        try:
            th = np.ascontiguousarray(ds.injection[None, :])
            st = np.empty((1, B.SCS_NSTATS))
            B.scs_evaluate_stats(h, th, st)
            dd = B.scs_data_norm(h)
            amp = np.array([ds.snr / np.sqrt(st[0, 2])])
            semi, coh = np.empty(1), np.empty(1)
            B.scs_loglike(h, st, amp, np.zeros(1), semi, coh)
            print("noise-free log L", semi, coh, "scale", dd)
            assert abs(semi[0]) < 1e-9 * dd and abs(coh[0]) < 1e-9 * dd
        finally:
            B.scs_ctx_destroy(h)


def test_distance_amplitude_and_coherent_loglike():
    """The coherent log-likelihood with the absolute amplitude from the
    luminosity distance (eqn:LogL_coherent; Sec 4: D_L is a 1/D_L prefactor
    of the amplitude): data carry the injection at its physical amplitude for
    a distance D_L*; the device amplitudes equal the oracle's, log L at the
    injected (theta, D_L, phase) against the oracle, and without noise log L
    peaks at D_L* (where it is 0) along a grid of distances."""
    base = D.lisa_small(seed=75, noise=False, snr=0.0)
    g, m, psd = base.grid, base.model, base.psd
    inj = base.injection
    h = O.template(g, m, inj)
    hh = D.inner(g, psd, h, h)
    a1 = float(O.distance_amplitude(inj[0], 1.0))
    dl_true = a1 * np.sqrt(hh) / 20.0  # SNR 20 at this distance
    for noise in (False, True):
        d = float(O.distance_amplitude(inj[0], dl_true)) * h
        if noise:
            d = d + synth.noise(psd, g.df, 76)
        ds = D.Dataset(g, m, psd, d, inj, 20.0, None, None)
        th = D.lisa_particles(6, seed=77)
        th[0] = inj
        dl = np.full(6, dl_true)
        dl[1] = -1.0  # invalid distance: NaN amplitude
        ctx = _ctx(ds, 8, G=16)
        try:
            amp = np.empty(6)
            B.scs_distance_amplitude(ctx, np.ascontiguousarray(th), dl, amp)
            ref_amp = O.distance_amplitude(th[:, 0], dl)
            assert np.isnan(amp[1]) and np.isnan(ref_amp[1])
            ok = np.isfinite(ref_amp)
            assert np.all(np.abs(amp[ok] / ref_amp[ok] - 1) < 1e-14), amp / ref_amp
            st = np.empty((6, B.SCS_NSTATS))
            B.scs_evaluate_stats(ctx, np.ascontiguousarray(th), st)
            dd = B.scs_data_norm(ctx)
            semi, coh = np.empty(6), np.empty(6)
            B.scs_loglike(ctx, st, np.nan_to_num(amp), np.zeros(6), semi, coh)
            rs = O.likelihood_stats(g, m, ds.d_ri, psd, th, 8, O.SEG_EQUAL_SNR, 16)
            ref_semi, ref_coh = O.loglike(O.data_norm(g, ds.d_ri, psd), rs, np.nan_to_num(ref_amp), np.zeros(6))
            scale = dd + np.nan_to_num(ref_amp) ** 2 * rs["hh"]
            e = np.abs(coh - ref_coh)[ok] / scale[ok]
            print(f"noise {noise}: coherent log L at the physical amplitude, max err {e.max():.3g}; "
                  f"log L(theta*, D_L*) = {coh[0]:.6g}")
            assert e.max() < 1e-9
            if not noise:
                assert abs(coh[0]) < 1e-9 * dd
                # log L along distances: its maximum sits at D_L*
                grid_dl = dl_true * np.linspace(0.8, 1.2, 41)
                a = np.empty(41)
                B.scs_distance_amplitude(ctx, np.ascontiguousarray(np.tile(inj, (41, 1))), grid_dl, a)
                _, c41 = np.empty(41), np.empty(41)
                B.scs_loglike(ctx, np.ascontiguousarray(np.tile(st[0], (41, 1))), a, np.zeros(41), None, c41)
                assert int(np.argmax(c41)) == 20, np.argmax(c41)
        finally:
            B.scs_ctx_destroy(ctx)
