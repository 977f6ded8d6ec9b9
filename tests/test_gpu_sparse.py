"""Parity of the sparse-grid template (Sec 4, waveform and response
paragraphs: waveform and response on a grid coarser than the FFT grid,
cubic-spline interpolated onto it) through the C ABI against the oracle's
sparse-grid mode: the template per bin, Upsilon_N in FP64 and mixed precision
for every response model, the one-, two- and three-node supports, a batched
launch beside per-bin contexts, and the 2^20-bin workload at full size with
the paper's stride of 1000 bins.

Tolerances: the template within 1e-10 of max|h| (node phases reduced in
double-double on both sides, spline arithmetic in FP64 here and in extended
precision in the oracle: about 1e-13 cycles at a stride of 1000), Upsilon_N
within 1e-9 (FP64) and 1e-5 (mixed) floored relative error (floor 2 N_eff),
supports and edges bit-exact except at a rounding tie of the oracle's
cumulative (tests/parity.py).  The edges keep the exact weights, so they are
those of the per-bin template.
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


def _sparse(m, S):
    return O.Model(pn_order=m.pn_order, response=m.response, support=m.support, t_obs=m.t_obs,
                   eccentric=m.eccentric, sparse_stride=S)


def _ctx(ds, model, N, mode=B.SCS_SEG_EQUAL_SNR, G=1):
    g = ds.grid
    h = B.scs_ctx_create(0)
    B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
    B.scs_set_model(h, model.pn_order, model.response, model.support, model.t_obs, eccentric=model.eccentric,
                    sparse_stride=model.sparse_stride)
    B.scs_define_segmentation(h, N, mode, G)
    return h


def _dataset(kind, noise=True, seed=61):
    if kind == "white":
        return D.white_small(K=4096, seed=seed, noise=noise)
    if kind == "lf":
        return D.lisa_small(seed=seed, noise=noise)
    if kind == "fd2":
        return D.lisa_small(seed=seed, noise=noise, response=O.RESP_LISA_FD, n_chan=2)
    if kind == "fd3":
        return D.lisa_small(seed=seed, noise=noise, response=O.RESP_LISA_FD, n_chan=3)
    if kind == "ecc":
        ds = D.lisa_small(seed=seed, noise=noise)
        m = ds.model
        em = O.Model(pn_order=m.pn_order, response=m.response, support=m.support, t_obs=m.t_obs, eccentric=1)
        inj = np.append(ds.injection, 0.05)
        return D.make(ds.grid, em, ds.psd, inj, ds.snr, seed, noise, None, None)
    raise KeyError(kind)


def _particles(ds, n, seed):
    if ds.grid.n_chan == 1:
        th = synth.single_channel_particles(n, seed)
        th[:2] = ds.injection
        return th
    th = D.lisa_particles(n, seed=seed)
    th[:3] = synth.near_injection(ds.injection[:7], 3, seed=seed + 1)
    if ds.model.eccentric:
        e0 = np.random.default_rng(seed + 2).uniform(0.005, 0.1, n)
        th = np.concatenate([th, e0[:, None]], axis=1)
    return th


@pytest.mark.parametrize("kind,S", [("white", 100), ("lf", 1000), ("lf", 128), ("fd2", 1000), ("fd3", 256),
                                    ("ecc", 1000)])
def test_sparse_template_matches_oracle(kind, S):
    ds = _dataset(kind, noise=False)
    ms = _sparse(ds.model, S)
    h = _ctx(ds, ms, 1)
    try:
        nch = ds.grid.n_chan
        for th in list(_particles(ds, 5, seed=62)):
            out = torch.empty((nch, ds.grid.K, 2), dtype=torch.float64, device="cuda")
            B.scs_waveform(h, torch.tensor(np.ascontiguousarray(th), device="cuda"), out)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            gc = got[..., 0] + 1j * got[..., 1]
            ref = O.template(ds.grid, ms, th)
            exact = O.template(ds.grid, ds.model, th)
            nz = np.abs(ref) > 0
            assert np.array_equal(nz, np.abs(gc) > 0), "supports differ"
            scale = np.abs(ref).max()
            err = np.abs(gc - ref)[nz].max() / scale
            interp = np.abs(ref - exact)[nz].max() / scale
            print(f"{kind}, S = {S}: sparse template max err / max|h| {err:.3g} "
                  f"(interpolation itself {interp:.3g})")
            assert err < 1e-10
            assert interp > 100 * err  # the spline, not the per-bin template
    finally:
        B.scs_ctx_destroy(h)


@pytest.mark.parametrize("kind,S,N,mode,G", [
    ("white", 100, 16, B.SCS_SEG_EQUAL_SNR, 1), ("lf", 1000, 1, B.SCS_SEG_EQUAL_SNR, 1),
    ("lf", 1000, 8, B.SCS_SEG_EQUAL_SNR, 16), ("lf", 300, 64, B.SCS_SEG_EQUAL_SNR, 1),
    ("lf", 1000, 37, B.SCS_SEG_UNIFORM, 1), ("fd2", 1000, 16, B.SCS_SEG_EQUAL_SNR, 16),
    ("fd3", 500, 8, B.SCS_SEG_EQUAL_SNR, 1), ("ecc", 1000, 8, B.SCS_SEG_EQUAL_SNR, 16)])
def test_sparse_upsilon_matches_oracle(kind, S, N, mode, G):
    ds = _dataset(kind, seed=63)
    ms = _sparse(ds.model, S)
    th = _particles(ds, 40, seed=64)
    th[4, 0] = -1.0  # invalid: NaN
    if ds.grid.n_chan > 1:
        th[5, 2] = 0.0195  # empty support: 0
    ref = O.evaluate(ds.grid, ms, ds.d_ri, ds.psd, th, N, mode, G, want_bounds=True)
    h = _ctx(ds, ms, N, mode, G)
    try:
        tht = torch.tensor(np.ascontiguousarray(th), device="cuda")
        u = torch.empty(th.shape[0], dtype=torch.float64, device="cuda")
        B.scs_evaluate(h, tht, u, B.SCS_PREC_FP64)
        torch.cuda.synchronize()
        got = u.cpu().numpy()
        assert np.isnan(got[4])
        if ds.grid.n_chan > 1:
            assert got[5] == 0.0
        sup, bnd = B.scs_last_bounds(h, th.shape[0], N)
        ok = np.isfinite(ref["ups"])
        assert np.array_equal(sup[ok], ref["support"][ok])
        PT.check_rows(ds, th, got, ref, bnd, G, PT.TOL64, mode, what=f"{kind} S={S} N={N} fp64", model=ms)
        B.scs_evaluate(h, tht, u, B.SCS_PREC_MIXED)
        torch.cuda.synchronize()
        PT.check_rows(ds, th, u.cpu().numpy(), ref, bnd, G, PT.TOLMIX, mode, what=f"{kind} S={S} N={N} mixed",
                      model=ms)
        # how far the interpolation moves the statistic on these short test
        # bands (coarse: a stride of S bins spans far more of the chirp here
        # than on the 2^20-bin band, where the full-size test below bounds it)
        exact = O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, th[ok], N, mode, G)["ups"]
        dif = PT.floored(got[ok], exact, PT.n_eff(ref["bounds"][ok]))
        print(f"{kind} S={S} N={N}: sparse vs per-bin template Upsilon, max floored difference {dif.max():.3g}")
        assert dif.max() > 0
    finally:
        B.scs_ctx_destroy(h)


def test_sparse_small_supports():
    """Supports of one, two and three nodes (the constant, the line, the
    parabola), among them supports of one and two bins: the template and
    Upsilon_N against the oracle."""
    ds = D.lisa_small(seed=65, noise=True)
    th = ds.injection.copy()
    for fl, S, t_obs in [(0.018999, 4096, 1e7), (0.01895, 512, 1e7), (0.0185, 1024, 1.0), (0.0185, 1000, 1000.0)]:
        th[2] = fl
        m = O.Model(pn_order=ds.model.pn_order, response=ds.model.response, support=ds.model.support, t_obs=t_obs)
        ms = _sparse(m, S)
        dsm = D.Dataset(ds.grid, m, ds.psd, ds.d, th, 0.0, None, None)
        ref = O.evaluate(dsm.grid, ms, dsm.d_ri, dsm.psd, th[None, :], 4, O.SEG_EQUAL_SNR, 1, want_bounds=True)
        h = _ctx(dsm, ms, 4)
        try:
            u = np.empty(1)
            B.scs_evaluate(h, np.ascontiguousarray(th[None, :]), u, B.SCS_PREC_FP64)
            sup, bnd = B.scs_last_bounds(h, 1, 4)
            k0, k1 = ref["support"][0]
            print(f"f_low {fl}, S {S}, T_obs {t_obs}: support {k1 - k0} bins, Upsilon {u[0]:.12g} "
                  f"oracle {ref['ups'][0]:.12g}")
            PT.check_rows(dsm, th[None, :], u, ref, bnd, 1, PT.TOL64, what=f"small support S={S}", model=ms)
            out = np.empty((2, ds.grid.K, 2))
            B.scs_waveform(h, np.ascontiguousarray(th), out)
            gc = out[..., 0] + 1j * out[..., 1]
            want = O.template(dsm.grid, ms, th)
            assert np.array_equal(np.abs(want) > 0, np.abs(gc) > 0)
            if np.abs(want).max() > 0:
                assert np.abs(gc - want).max() <= 1e-10 * np.abs(want).max()
        finally:
            B.scs_ctx_destroy(h)


def test_sparse_in_a_batch():
    """A sparse-grid context inside a batched launch with a per-bin context
    of the same data: every item equals its solo evaluation bit for bit."""
    ds = D.lisa_small(seed=66)
    ms = _sparse(ds.model, 1000)
    th = _particles(ds, 300, seed=67)
    ha = _ctx(ds, ms, 16, G=16)
    hb = _ctx(ds, ds.model, 8, G=16)
    try:
        tht = torch.tensor(np.ascontiguousarray(th), device="cuda")
        for prec in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
            solo_a = torch.empty(th.shape[0], dtype=torch.float64, device="cuda")
            solo_b = torch.empty_like(solo_a)
            B.scs_evaluate(ha, tht, solo_a, prec)
            B.scs_evaluate(hb, tht, solo_b, prec)
            ba = torch.empty_like(solo_a)
            bb = torch.empty_like(solo_a)
            B.scs_evaluate_batched([(ha, 16, tht, ba), (hb, 8, tht, bb)], prec)
            torch.cuda.synchronize()
            assert torch.equal(ba, solo_a) and torch.equal(bb, solo_b)
            assert not torch.equal(solo_a[:50], solo_b[:50])
        ref = O.evaluate(ds.grid, ms, ds.d_ri, ds.psd, th[:12], 16, O.SEG_EQUAL_SNR, 16, want_bounds=True)
        B.scs_evaluate(ha, tht, solo_a, B.SCS_PREC_FP64)
        torch.cuda.synchronize()
        _, bnd = B.scs_last_bounds(ha, th.shape[0], 16)
        PT.check_rows(ds, th[:12], solo_a.cpu().numpy()[:12], ref, bnd[:12], 16, PT.TOL64, what="batched sparse",
                      model=ms)
    finally:
        B.scs_ctx_destroy(ha)
        B.scs_ctx_destroy(hb)


def test_sparse_lisa1m_full_size_sampled():
    """The 2^20-bin A+E workload at full size (10^4 particles, N = 1024,
    G = 1024) with the paper's stride of 1000 bins; the oracle recomputes a
    seeded sample of particles one by one."""
    w = synth.workload("lisa1m")
    g = O.Grid(w.grid.K, w.grid.k0, w.grid.df, 2)
    m = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=w.grid.t_obs)
    ds = D.make(g, m, synth.psd_arrays(w), w.injection, w.snr, w.seed, True, w.prior_lo, w.prior_hi)
    ms = _sparse(m, 1000)
    theta = synth.workload_particles(w)
    theta[:2] = synth.near_injection(w.injection, 2, seed=5, lo=w.prior_lo, hi=w.prior_hi)
    N = w.N
    h = _ctx(ds, ms, N, B.SCS_SEG_EQUAL_SNR, w.G)
    try:
        tht = torch.tensor(theta, device="cuda")
        u = torch.empty(theta.shape[0], dtype=torch.float64, device="cuda")
        B.scs_evaluate(h, tht, u, B.SCS_PREC_FP64)
        torch.cuda.synchronize()
        got = u.cpu().numpy()
        sup, bnd = B.scs_last_bounds(h, theta.shape[0], N)
        B.scs_evaluate(h, tht, u, B.SCS_PREC_MIXED)
        torch.cuda.synchronize()
        gm = u.cpu().numpy()
        assert np.all(np.isfinite(got)) and np.all(got >= 0)
        idx = np.concatenate([[0, 1], np.random.default_rng(7).choice(np.arange(2, len(theta)), 4, replace=False)])
        ref = O.evaluate(ds.grid, ms, ds.d_ri, ds.psd, theta[idx], N, O.SEG_EQUAL_SNR, w.G, want_bounds=True)
        assert np.array_equal(sup[idx], ref["support"])
        PT.check_rows(ds, theta[idx], got[idx], ref, bnd[idx], w.G, PT.TOL64, what="lisa1m sparse fp64", model=ms)
        PT.check_rows(ds, theta[idx], gm[idx], ref, bnd[idx], w.G, PT.TOLMIX, what="lisa1m sparse mixed", model=ms)
        ok = got > 0
        eall = PT.floored(gm[ok], got[ok], PT.n_eff(bnd[ok]))
        print("sparse mixed vs fp64, all 10^4 particles: median", np.median(eall), "max", eall.max())
        assert eall.max() < PT.TOLMIX
        # at the paper's stride on this band the interpolation (1e-6 cycles of
        # phase) moves the statistic at second order only
        exact = O.evaluate(ds.grid, m, ds.d_ri, ds.psd, theta[idx], N, O.SEG_EQUAL_SNR, w.G)["ups"]
        dif = PT.floored(got[idx], exact, PT.n_eff(ref["bounds"]))
        print("lisa1m: sparse vs per-bin template Upsilon, max floored difference", dif.max())
        assert 0 < dif.max() < 1e-6
    finally:
        B.scs_ctx_destroy(h)


def test_sparse_noalloc_equals_evaluate():
    """The evaluation without allocation lays the node records out in its
    static scratch too: two calls in a row (the second smaller) equal
    scs_evaluate bit for bit."""
    ds = D.lisa_small(seed=68)
    ms = _sparse(ds.model, 1000)
    h = _ctx(ds, ms, 16, G=16)
    try:
        for P, seed in ((300, 69), (50, 70)):
            print(f"sparse noalloc P {P}", flush=True)
            th = torch.tensor(np.ascontiguousarray(_particles(ds, P, seed)), device="cuda")
            u_ref = torch.empty(P, dtype=torch.float64, device="cuda")
            u_na = torch.full((P,), -7.0, dtype=torch.float64, device="cuda")
            for prec in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
                B.scs_evaluate(h, th, u_ref, prec)
                B.scs_evaluate_noalloc(h, th, u_na, prec)
                torch.cuda.synchronize()
                assert torch.equal(u_na, u_ref)
    finally:
        B.scs_ctx_destroy(h)


def test_unresolved_theta_is_nan_per_bin_and_finite_on_the_sparse_grid():
    """The per-bin template needs a polynomial block length whose remainder
    bounds hold; a slowly chirping low-mass source on a coarse grid has none
    (here Mc = 4 on the 1e-7 Hz grid: its SPA time moves ~3e4 s per bin, so
    even an 8-bin block leaves the response's fourth orbital harmonic above
    the 1e-11 bound).  Such a theta gives NaN and is counted by
    scs_ctx_stats; the sparse-grid template expands nothing in blocks and
    evaluates it like any other (against the oracle)."""
    ds = D.lisa_small(seed=71)
    th = np.tile(ds.injection, (3, 1))
    th[1, 0] = 4.0  # unresolved
    th[2, 0] = 27.5
    N = 4
    h = _ctx(ds, ds.model, N, G=16)
    try:
        B.scs_ctx_stats(h, reset=True)
        u = np.empty(3)
        for prec in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
            B.scs_evaluate(h, np.ascontiguousarray(th), u, prec)
            assert np.isnan(u[1]) and np.all(np.isfinite(u[[0, 2]])), (prec, u)
        _, _, unresolved = B.scs_ctx_stats(h, reset=True)
        assert unresolved == 2  # one particle, two evaluations
    finally:
        B.scs_ctx_destroy(h)
    ms = _sparse(ds.model, 200)
    ref = O.evaluate(ds.grid, ms, ds.d_ri, ds.psd, th, N, O.SEG_EQUAL_SNR, 16, want_bounds=True)
    h = _ctx(ds, ms, N, G=16)
    try:
        u = np.empty(3)
        B.scs_evaluate(h, np.ascontiguousarray(th), u, B.SCS_PREC_FP64)
        _, bnd = B.scs_last_bounds(h, 3, N)
        _, _, unresolved = B.scs_ctx_stats(h, reset=True)
        assert unresolved == 0
        print("unresolved per bin, sparse grid:", u, "oracle", ref["ups"])
        PT.check_rows(ds, th, u, ref, bnd, 16, PT.TOL64, what="unresolved theta on the sparse grid", model=ms)
    finally:
        B.scs_ctx_destroy(h)
