"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: FP64 path within 1e-9 floored relative error,
|U_gpu - U_ref| / max(U_ref, 2 N_eff), N_eff the non-empty segments of the
row; mixed path within 1e-5 on the same measure.  Segment edges and supports
are integers and must match exactly; an equal-[h|h] edge may differ only at a
rounding tie of the oracle's cumulative, and such a row is then compared with
the oracle on the GPU's edges (tests/parity.py).
"""
import functools

import numpy as np
import pytest

import oracle as O
import synth
from tests import datasets as D
from tests import parity as PT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_13170_amd import B  # noqa: E402

TOL64 = PT.TOL64
TOLMIX = PT.TOLMIX


class Ctx:
    def __init__(self, ds, N, mode=B.SCS_SEG_EQUAL_SNR, G=1, edges=None, block_len=0):
        self.ds = ds
        self.N = N
        self.h = B.scs_ctx_create(0)
        g = ds.grid
        B.scs_load_data(self.h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
        m = ds.model
        B.scs_set_model(self.h, m.pn_order, m.response, m.support, m.t_obs, block_len)
        B.scs_define_segmentation(self.h, N, mode, G, edges)

    def eval(self, theta, prec=B.SCS_PREC_FP64, seg=False):
        th = torch.tensor(np.ascontiguousarray(theta), device="cuda")
        ups = torch.empty(th.shape[0], dtype=torch.float64, device="cuda")
        sg = torch.empty((th.shape[0], self.N, 3), dtype=torch.float64, device="cuda") if seg else None
        B.scs_evaluate(self.h, th, ups, prec, sg)
        torch.cuda.synchronize()
        return ups.cpu().numpy(), (sg.cpu().numpy() if seg else None)

    def close(self):
        B.scs_ctx_destroy(self.h)


def _ref(ds, theta, N, mode=O.SEG_EQUAL_SNR, G=1, edges=None, seg=False):
    return O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, theta, N, mode, G, edges, want_seg=seg,
                      want_bounds=True)


def test_waveform_matches_oracle_white16k():
    ds = D.white16k()
    c = Ctx(ds, 1)
    try:
        for th in (ds.injection, synth.single_channel_particles(2, 5)[1]):
            h = torch.empty((1, ds.grid.K, 2), dtype=torch.float64, device="cuda")
            B.scs_waveform(c.h, torch.tensor(th, device="cuda"), h)
            torch.cuda.synchronize()
            got = h.cpu().numpy()
            ref = O.template(ds.grid, ds.model, th)
            gc = got[..., 0] + 1j * got[..., 1]
            rel = np.abs(gc - ref) / np.abs(ref)
            print("white16k template max rel err", rel.max())
            assert rel.max() < 1e-10
    finally:
        c.close()


def test_waveform_matches_oracle_lisa_small():
    ds = D.lisa_small(noise=False)
    c = Ctx(ds, 1)
    try:
        ths = [ds.injection] + list(D.lisa_particles(3, seed=77))
        for th in ths:
            h = torch.empty((2, ds.grid.K, 2), dtype=torch.float64, device="cuda")
            B.scs_waveform(c.h, torch.tensor(np.ascontiguousarray(th), device="cuda"), h)
            torch.cuda.synchronize()
            got = h.cpu().numpy()
            gc = got[..., 0] + 1j * got[..., 1]
            ref = O.template(ds.grid, ds.model, th)
            nz = np.abs(ref) > 0
            assert np.array_equal(nz, np.abs(gc) > 0), "supports differ"
            scale = np.abs(ref).max()
            err = np.abs(gc - ref)[nz].max() / scale
            print("lisa template max err / max|h|", err)
            assert err < 1e-10
    finally:
        c.close()


def test_upsilon_white16k_fp64_and_mixed():
    """The 16384-bin single-channel workload in full: 64 particles, N = 16."""
    w = synth.workload("white16k")
    ds = D.white16k()
    theta = synth.workload_particles(w)
    ref = _ref(ds, theta, 16, seg=True)
    c = Ctx(ds, 16)
    try:
        got, seg = c.eval(theta, seg=True)
        sup, bnd = B.scs_last_bounds(c.h, theta.shape[0], 16)
        assert np.array_equal(bnd, ref["bounds"])
        assert np.array_equal(sup, ref["support"])
        PT.check_rows(ds, theta, got, ref, bnd, 1, TOL64, what="white16k fp64")
        rs = ref["seg"]
        zerr = np.abs(seg[..., :2] - rs[..., :2]).max() / np.abs(rs[..., :2]).max()
        herr = np.abs(seg[..., 2] / rs[..., 2] - 1).max()
        assert zerr < 1e-9 and herr < 1e-12
        gm, _ = c.eval(theta, prec=B.SCS_PREC_MIXED)
        PT.check_rows(ds, theta, gm, ref, bnd, 1, TOLMIX, what="white16k mixed")
    finally:
        c.close()


@pytest.mark.parametrize("N,mode,G", [(1, O.SEG_EQUAL_SNR, 1), (8, O.SEG_EQUAL_SNR, 16),
                                      (64, O.SEG_EQUAL_SNR, 1), (37, O.SEG_UNIFORM, 1)])
def test_upsilon_lisa_small(N, mode, G):
    ds = D.lisa_small(seed=3)
    th = D.lisa_particles(40, seed=11)
    th[:4] = synth.near_injection(ds.injection, 4, seed=2)
    ref = _ref(ds, th, N, mode, G)
    c = Ctx(ds, N, mode, G)
    try:
        got, _ = c.eval(th)
        sup, bnd = B.scs_last_bounds(c.h, th.shape[0], N)
        assert np.array_equal(sup, ref["support"])
        PT.check_rows(ds, th, got, ref, bnd, G, TOL64, mode, what=f"lisa_small N={N} fp64")
        gm, _ = c.eval(th, prec=B.SCS_PREC_MIXED)
        PT.check_rows(ds, th, gm, ref, bnd, G, TOLMIX, mode, what=f"lisa_small N={N} mixed")
    finally:
        c.close()


def test_edge_cases_lisa_small():
    ds = D.lisa_small(seed=4)
    th = np.tile(ds.injection, (70, 1))
    th[1, 0] = -1.0        # invalid chirp mass
    th[2, 1] = 0.3         # eta > 1/4
    th[3, 2] = 0.0195      # support empty (f_low above the band)
    th[4, 2] = 0.018999    # 10 bins of support: 22 of the 32 segments empty
    th[5, 2] = 0.0189975   # 24 bins: 8 empty segments
    th[6, 2] = 0.01895     # 499 bins
    th[7:, :] = D.lisa_particles(63, seed=8)
    N = 32
    ref = _ref(ds, th, N, O.SEG_EQUAL_SNR, 1, seg=True)
    c = Ctx(ds, N, B.SCS_SEG_EQUAL_SNR, 1)
    try:
        got, seg = c.eval(th, seg=True)
        assert np.isnan(got[1]) and np.isnan(got[2])
        assert got[3] == 0.0
        ok = ~np.isnan(ref["ups"])
        sup, bnd = B.scs_last_bounds(c.h, th.shape[0], N)
        assert np.array_equal(sup, ref["support"])
        PT.check_rows(ds, th, got, ref, bnd, 1, TOL64, what="edge cases fp64")
        # per-segment (Z, H): empty segments (particles 4 and 5 have runs of
        # them) exactly zero, the others against the oracle (rows with the
        # oracle's edges; a tied row was checked on its own edges above)
        rows = np.flatnonzero(ok & np.all(bnd == ref["bounds"], axis=1))
        assert 4 in rows and 5 in rows
        rs = ref["seg"]
        empty = bnd[:, 1:] == bnd[:, :-1]
        assert empty[4].sum() == 22 and empty[5].sum() == 8
        for p in rows:
            assert np.all(seg[p][empty[p]] == 0.0)
            full = ~empty[p]
            if not full.any():  # empty support
                continue
            zscale = np.abs(rs[p][full, :2]).max()
            assert np.abs(seg[p][full, :2] - rs[p][full, :2]).max() <= 1e-9 * zscale
            # H carries |R|^2 of the interpolated response: the block length is
            # chosen for 1e-11 relative on R, so 2e-11 on |R|^2 (seen as such on
            # one-bin segments, where nothing averages it down)
            assert np.abs(seg[p][full, 2] / rs[p][full, 2] - 1.0).max() < 5e-11
        # determinism: bitwise identical on a second run
        got2, _ = c.eval(th)
        assert np.array_equal(got[ok], got2[ok])
        # P = 0 is a no-op
        B.scs_evaluate(c.h, torch.empty((0, 7), dtype=torch.float64, device="cuda"),
                       torch.empty(0, dtype=torch.float64, device="cuda"))
    finally:
        c.close()


def test_maximum_segment_count():
    """N at its documented maximum (2^20 segments over a support of a few
    thousand bins: nearly every segment empty or one bin long) against the
    oracle, and N one above it rejected."""
    ds = D.lisa_small(seed=4)
    th = D.lisa_particles(8, seed=9)
    th[0] = ds.injection
    N = B.SCS_MAX_SEGMENTS
    ref = _ref(ds, th, N, O.SEG_EQUAL_SNR, 1)
    c = Ctx(ds, N, B.SCS_SEG_EQUAL_SNR, 1)
    try:
        got, _ = c.eval(th)
        sup, bnd = B.scs_last_bounds(c.h, th.shape[0], N)
        assert np.array_equal(sup, ref["support"])
        print("N = 2^20: non-empty segments per row", PT.n_eff(ref["bounds"]))
        PT.check_rows(ds, th, got, ref, bnd, 1, TOL64, what="N = 2^20 fp64")
        gm, _ = c.eval(th, B.SCS_PREC_MIXED)
        PT.check_rows(ds, th, gm, ref, bnd, 1, TOLMIX, what="N = 2^20 mixed")
        with pytest.raises(B.ScsError):
            B.scs_define_segmentation(c.h, N + 1, B.SCS_SEG_EQUAL_SNR, 1)
    finally:
        c.close()


@functools.lru_cache(maxsize=1)
def _lisa1m_dataset():
    w = synth.workload("lisa1m")
    g = O.Grid(w.grid.K, w.grid.k0, w.grid.df, 2)
    m = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=w.grid.t_obs)
    psd = synth.psd_arrays(w)
    return w, D.make(g, m, psd, w.injection, w.snr, w.seed, True, w.prior_lo, w.prior_hi)


def test_upsilon_lisa1m_full_size_sampled():
    """The 2^20-bin A+E workload at its full size (10^4 particles, N = 1024,
    G = 1024) in the launch configuration the benchmark uses; the oracle
    recomputes a seeded sample of particles one by one."""
    w, ds = _lisa1m_dataset()
    theta = synth.workload_particles(w)
    theta[:2] = synth.near_injection(w.injection, 2, seed=5, lo=w.prior_lo, hi=w.prior_hi)
    N = w.N
    c = Ctx(ds, N, B.SCS_SEG_EQUAL_SNR, w.G)
    try:
        got, _ = c.eval(theta)
        sup, bnd = B.scs_last_bounds(c.h, theta.shape[0], N)
        gm, _ = c.eval(theta, prec=B.SCS_PREC_MIXED)
        assert np.all(np.isfinite(got)) and np.all(got >= 0)
        idx = np.concatenate([[0, 1], np.random.default_rng(3).choice(np.arange(2, len(theta)), 6, replace=False)])
        ref = _ref(ds, theta[idx], N, O.SEG_EQUAL_SNR, w.G)
        assert np.array_equal(sup[idx], ref["support"])
        PT.check_rows(ds, theta[idx], got[idx], ref, bnd[idx], w.G, TOL64, what="lisa1m sampled fp64")
        PT.check_rows(ds, theta[idx], gm[idx], ref, bnd[idx], w.G, TOLMIX, what="lisa1m sampled mixed")
        print("Upsilon near injection", got[:2], "oracle", ref["ups"][:2])
        # mixed against FP64 over every particle (same boundaries by construction)
        ok = got > 0
        eall = PT.floored(gm[ok], got[ok], PT.n_eff(bnd[ok]))
        print("mixed vs fp64, all 10^4 particles: median", np.median(eall), "p99", np.quantile(eall, 0.99),
              "max", eall.max())
        assert eall.max() < TOLMIX
    finally:
        c.close()


def test_growing_block_lengths_lisa1m():
    """Blocks that grow along the support (up to 2048 bins) against blocks
    capped at 512 bins (about the length this prior box's support starts
    allow, so they can hardly grow): both expand the template within the same
    bounds, so over all 10^4 particles of the 2^20-bin workload the two agree
    far inside the FP64 tolerance, and the mixed path within its own."""
    w, ds = _lisa1m_dataset()
    theta = synth.workload_particles(w)
    N = w.N
    c1 = Ctx(ds, N, B.SCS_SEG_EQUAL_SNR, w.G)
    c2 = Ctx(ds, N, B.SCS_SEG_EQUAL_SNR, w.G, block_len=512)
    try:
        g1, _ = c1.eval(theta)
        g2, _ = c2.eval(theta)
        _, bnd = B.scs_last_bounds(c1.h, theta.shape[0], N)
        _, bnd2 = B.scs_last_bounds(c2.h, theta.shape[0], N)
        assert np.array_equal(bnd, bnd2)
        assert np.all(np.isfinite(g1)) and np.all(np.isfinite(g2))
        e = PT.floored(g1, g2, PT.n_eff(bnd))
        print("fp64, growing vs 512-bin blocks: median", np.median(e), "max", e.max())
        assert e.max() < 1e-11
        m1, _ = c1.eval(theta, prec=B.SCS_PREC_MIXED)
        m2, _ = c2.eval(theta, prec=B.SCS_PREC_MIXED)
        em = PT.floored(m1, g2, PT.n_eff(bnd))
        print("mixed with growing blocks vs fp64 with 512-bin blocks: max", em.max(),
              "; mixed with 512-bin blocks:", PT.floored(m2, g2, PT.n_eff(bnd)).max())
        assert em.max() < TOLMIX
    finally:
        c1.close()
        c2.close()
