"""Batched evaluation of uneven swarms (one fused persistent launch per
channel count) and its HIP-graph replay equal the solo evaluations bit for
bit, and agree with the oracle."""
import numpy as np
import pytest

import oracle as O
import synth
from tests import datasets as D
from tests import parity as PT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_13170_amd import B  # noqa: E402


def _ctx(ds, N=1, G=16):
    g = ds.grid
    h = B.scs_ctx_create(0)
    B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
    m = ds.model
    B.scs_set_model(h, m.pn_order, m.response, m.support, m.t_obs)
    B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, G)
    return h


def test_batched_and_graph_equal_solo():
    lisa = D.lisa_small(seed=9)
    white = D.white16k()
    hl, hw = _ctx(lisa), _ctx(white, G=1)
    try:
        wth = synth.workload_particles(synth.workload("white16k"))
        # (context, dataset, N, P, theta)
        shapes = [(hl, lisa, 256, 700, D.lisa_particles(700, seed=100)),
                  (hw, white, 16, 64, wth),
                  (hl, lisa, 64, 300, D.lisa_particles(300, seed=101)),
                  (hl, lisa, 16, 129, D.lisa_particles(129, seed=102)),
                  (hw, white, 4, 33, wth[:33]),
                  (hl, lisa, 1, 64, D.lisa_particles(64, seed=103))]
        items = []
        for h, ds, N, P, th in shapes:
            items.append((h, N, torch.tensor(np.ascontiguousarray(th), device="cuda"),
                          torch.full((P,), -1.0, dtype=torch.float64, device="cuda")))
        for prec in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
            B.scs_evaluate_batched(items, prec)
            torch.cuda.synchronize()
            batched = [it[3].cpu().numpy().copy() for it in items]
            for (h, ds, N, P, th), bv in zip(shapes, batched):
                B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, 1 if ds is white else 16)
                u = torch.empty(P, dtype=torch.float64, device="cuda")
                B.scs_evaluate(h, torch.tensor(np.ascontiguousarray(th), device="cuda"), u, prec)
                torch.cuda.synchronize()
                assert np.array_equal(u.cpu().numpy(), bv), (N, P, prec)
            if prec == B.SCS_PREC_FP64:
                # oracle spot check on two items of different channel counts
                # (edges from the solo evaluation of the same particles, which
                # gave the batched values bit for bit)
                for k in (0, 1):
                    h, ds, N, P, th = shapes[k]
                    G = 1 if ds is white else 16
                    ref = O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, th[:6], N, O.SEG_EQUAL_SNR, G,
                                     want_bounds=True)
                    B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, G)
                    u = torch.empty(6, dtype=torch.float64, device="cuda")
                    B.scs_evaluate(h, torch.tensor(np.ascontiguousarray(th[:6]), device="cuda"), u, prec)
                    _, bnd = B.scs_last_bounds(h, 6, N)
                    PT.check_rows(ds, th[:6], batched[k][:6], ref, bnd, G, PT.TOL64,
                                  what=f"batched vs oracle, item {k}")
            graph = B.scs_graph_create(items, prec)
            for rep in range(3):
                for it in items:
                    it[3].fill_(-1.0)
                torch.cuda.synchronize()
                B.scs_graph_launch(graph)
                torch.cuda.synchronize()
                for it, bv in zip(items, batched):
                    assert np.array_equal(it[3].cpu().numpy(), bv), rep
            B.scs_graph_destroy(graph)
    finally:
        B.scs_ctx_destroy(hl)
        B.scs_ctx_destroy(hw)


def test_graph_keeps_its_workspaces():
    """A graph owns the workspaces its captured kernels use: batched calls
    and PSO-sized evaluations of larger swarms and segment counts on the same
    context (which grow the context's own workspaces) leave its replays
    intact; a change of the context's segmentation makes the next replay fail
    with ESTATE instead of replaying stale state."""
    lisa = D.lisa_small(seed=25)
    h = _ctx(lisa)
    try:
        th_small = [D.lisa_particles(100, seed=120), D.lisa_particles(64, seed=121)]
        items = [(h, N, torch.tensor(th, device="cuda"), torch.full((th.shape[0],), -1.0, dtype=torch.float64,
                                                                    device="cuda"))
                 for N, th in zip((16, 4), th_small)]
        graph = B.scs_graph_create(items, B.SCS_PREC_FP64)
        B.scs_graph_launch(graph)
        torch.cuda.synchronize()
        first = [it[3].cpu().numpy().copy() for it in items]
        # bigger work on the same context: its workspaces grow (reallocate)
        big = [(h, 256, torch.tensor(D.lisa_particles(3000, seed=122), device="cuda"),
                torch.empty(3000, dtype=torch.float64, device="cuda")),
               (h, 64, torch.tensor(D.lisa_particles(2000, seed=123), device="cuda"),
                torch.empty(2000, dtype=torch.float64, device="cuda"))]
        B.scs_evaluate_batched(big, B.SCS_PREC_FP64)
        u = torch.empty(3000, dtype=torch.float64, device="cuda")
        B.scs_evaluate(h, big[0][2], u)
        torch.cuda.synchronize()
        for rep in range(2):
            for it in items:
                it[3].fill_(-1.0)
            torch.cuda.synchronize()
            B.scs_graph_launch(graph)
            torch.cuda.synchronize()
            for it, f in zip(items, first):
                assert np.array_equal(it[3].cpu().numpy(), f), rep
        B.scs_define_segmentation(h, 8, B.SCS_SEG_EQUAL_SNR, 16)
        with pytest.raises(B.ScsError) as ei:
            B.scs_graph_launch(graph)
        assert ei.value.code == B.SCS_ESTATE
        B.scs_graph_destroy(graph)
    finally:
        B.scs_ctx_destroy(h)


def test_batch_mixes_response_models():
    """One batched call (and its graph) over contexts of every kernel
    instantiation: low-frequency A+E, full-response A+E and A+E+T, one
    channel, and an eccentric low-frequency context (8-entry theta rows);
    each item equals its solo evaluation bit for bit."""
    lf = D.lisa_small(seed=31)
    fd = D.lisa_small(seed=32, response=O.RESP_LISA_FD)
    fd3 = D.lisa_small(seed=33, response=O.RESP_LISA_FD, n_chan=3)
    white = D.white16k()
    hl, hf, hw, h3 = _ctx(lf), _ctx(fd), _ctx(white, G=1), _ctx(fd3)
    he = B.scs_ctx_create(0)
    try:
        g = lf.grid
        B.scs_load_data(he, np.ascontiguousarray(lf.d_ri), np.ascontiguousarray(lf.psd), g.k0 * g.df, g.df)
        B.scs_set_model(he, 7, lf.model.response, lf.model.support, lf.model.t_obs, eccentric=1)
        B.scs_define_segmentation(he, 1, B.SCS_SEG_EQUAL_SNR, 16)
        th_e = np.concatenate([D.lisa_particles(90, seed=107), np.linspace(0.0, 0.1, 90)[:, None]], axis=1)
        wth = synth.workload_particles(synth.workload("white16k"))
        shapes = [(hf, 16, 16, D.lisa_particles(200, seed=104)),
                  (hl, 16, 8, D.lisa_particles(150, seed=105)),
                  (hw, 1, 4, wth[:40]),
                  (he, 16, 5, th_e),
                  (h3, 16, 12, D.lisa_particles(110, seed=108)),
                  (hf, 16, 1, D.lisa_particles(70, seed=106))]
        items = [(h, N, torch.tensor(np.ascontiguousarray(th), device="cuda"),
                  torch.full((th.shape[0],), -1.0, dtype=torch.float64, device="cuda")) for h, G, N, th in shapes]
        for prec in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
            B.scs_evaluate_batched(items, prec)
            torch.cuda.synchronize()
            batched = [it[3].cpu().numpy().copy() for it in items]
            for (h, G, N, th), bv in zip(shapes, batched):
                assert np.all(np.isfinite(bv))
                B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, G)
                u = torch.empty(th.shape[0], dtype=torch.float64, device="cuda")
                B.scs_evaluate(h, torch.tensor(np.ascontiguousarray(th), device="cuda"), u, prec)
                torch.cuda.synchronize()
                assert np.array_equal(u.cpu().numpy(), bv), (N, th.shape, prec)
            graph = B.scs_graph_create(items, prec)
            for it in items:
                it[3].fill_(-1.0)
            torch.cuda.synchronize()
            B.scs_graph_launch(graph)
            torch.cuda.synchronize()
            for it, bv in zip(items, batched):
                assert np.array_equal(it[3].cpu().numpy(), bv)
            B.scs_graph_destroy(graph)
        # the full-response item against the oracle
        ref = O.evaluate(fd.grid, fd.model, fd.d_ri, fd.psd, shapes[0][3][:5], 16, O.SEG_EQUAL_SNR, 16)
        B.scs_evaluate_batched(items, B.SCS_PREC_FP64)
        torch.cuda.synchronize()
        got = items[0][3].cpu().numpy()[:5]
        assert np.max(np.abs(got - ref["ups"]) / np.maximum(np.abs(ref["ups"]), 32.0)) < 1e-9
    finally:
        for h in (hl, hf, hw, he, h3):
            B.scs_ctx_destroy(h)


def test_batched_hierarchy_full_size_sampled():
    """The configuration `bench.py --mode batched` times, at full size: the six
    swarms of the hierarchy, (N, P) = (4096, 16384) ... (1, 128), on the
    2^20-bin A+E data (G = 1024) in one graph-captured batched launch; two
    particles of every level recomputed by the oracle, FP64 and mixed."""
    w = synth.workload("lisa1m")
    g = O.Grid(w.grid.K, w.grid.k0, w.grid.df, 2)
    m = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=w.grid.t_obs)
    psd = synth.psd_arrays(w)
    ds = D.make(g, m, psd, w.injection, w.snr, w.seed, True, w.prior_lo, w.prior_hi)
    h = B.scs_ctx_create(0)
    try:
        B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(psd), g.k0 * g.df, g.df)
        B.scs_set_model(h, 7, m.response, m.support, m.t_obs)
        B.scs_define_segmentation(h, w.N, B.SCS_SEG_EQUAL_SNR, w.G)
        thetas = [synth.particles(w.prior_lo, w.prior_hi, P, w.seed + 700 + i)
                  for i, (N, P) in enumerate(synth.LADDER_SWARMS)]
        items = [(h, N, torch.tensor(th, device="cuda"), torch.empty(P, dtype=torch.float64, device="cuda"))
                 for (N, P), th in zip(synth.LADDER_SWARMS, thetas)]
        got = {}
        for prec in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
            graph = B.scs_graph_create(items, prec)
            B.scs_graph_launch(graph)
            torch.cuda.synchronize()
            got[prec] = [it[3].cpu().numpy().copy() for it in items]
            B.scs_graph_destroy(graph)
        rng = np.random.default_rng(12)
        worst64 = worstmx = 0.0
        for lvl, ((N, P), th) in enumerate(zip(synth.LADDER_SWARMS, thetas)):
            assert np.all(np.isfinite(got[B.SCS_PREC_FP64][lvl]))
            idx = rng.choice(P, 2, replace=False)
            ref = O.evaluate(g, m, ds.d_ri, psd, th[idx], N, O.SEG_EQUAL_SNR, w.G, want_bounds=True)
            # the sampled particles' edges, from a solo evaluation (edges are
            # per particle; batched values equal solo ones bit for bit)
            B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, w.G)
            B.scs_evaluate(h, torch.tensor(np.ascontiguousarray(th[idx]), device="cuda"),
                           torch.empty(2, dtype=torch.float64, device="cuda"))
            _, bnd = B.scs_last_bounds(h, 2, N)
            e64 = PT.check_rows(ds, th[idx], got[B.SCS_PREC_FP64][lvl][idx], ref, bnd, w.G, PT.TOL64,
                                what=f"hierarchy N={N} P={P} fp64")
            emx = PT.check_rows(ds, th[idx], got[B.SCS_PREC_MIXED][lvl][idx], ref, bnd, w.G, PT.TOLMIX,
                                what=f"hierarchy N={N} P={P} mixed")
            worst64, worstmx = max(worst64, e64), max(worstmx, emx)
        print(f"batched hierarchy, 2^20 bins: fp64 sampled max floored rel err {worst64:.3g}, mixed {worstmx:.3g}")
    finally:
        B.scs_ctx_destroy(h)
