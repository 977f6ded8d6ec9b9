"""The request loop: requests of two searches (different channel counts,
segment counts, swarm sizes and precisions) submitted while others run are
admitted within the slot and HBM limits, batched, and each result equals the
evaluation of the same particles alone, bit for bit."""
import time

import numpy as np
import pytest

import synth
from tests import datasets as D
from tests import parity as PT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_13170_amd import B  # noqa: E402


def _ctx(ds, G):
    g = ds.grid
    h = B.scs_ctx_create(0)
    B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
    m = ds.model
    B.scs_set_model(h, m.pn_order, m.response, m.support, m.t_obs)
    B.scs_define_segmentation(h, 1, B.SCS_SEG_EQUAL_SNR, G)
    return h


def test_served_results_equal_alone():
    lisa, white = D.lisa_small(seed=21), D.white16k()
    hl, hw = _ctx(lisa, 16), _ctx(white, 1)
    wth = synth.workload_particles(synth.workload("white16k"))
    rng = np.random.default_rng(5)
    reqs = []
    for r in range(24):
        if r % 3 == 2:
            P = int(rng.integers(8, 65))
            reqs.append(dict(h=hw, G=1, N=int(rng.choice([1, 4, 16])), th=wth[:P].copy(),
                             prec=B.SCS_PREC_FP64 if r % 2 else B.SCS_PREC_MIXED))
        else:
            P = int(rng.integers(16, 400))
            reqs.append(dict(h=hl, G=16, N=int(rng.choice([1, 8, 64, 256])),
                             th=D.lisa_particles(P, seed=300 + r),
                             prec=B.SCS_PREC_FP64 if r % 2 else B.SCS_PREC_MIXED))
    try:
        fp = max(B.scs_footprint(q["h"], q["th"].shape[0], q["N"], q["prec"]) for q in reqs)
        budget = 3 * (fp + 8 * 8 * 400)
        srv = B.scs_server_create(0, max_inflight=4, hbm_budget=budget, n_streams=2)
        try:
            ids = {}
            for k, q in enumerate(reqs):
                q["ups"] = np.full(q["th"].shape[0], -1.0)
                ids[B.scs_server_submit(srv, q["h"], q["N"], q["th"], q["ups"], q["prec"])] = k
                if k % 5 == 4:
                    time.sleep(0.002)  # later requests arrive while earlier ones run
            done = []
            t_end = time.time() + 60
            while len(done) < len(reqs) and time.time() < t_end:
                done += B.scs_server_poll(srv, wait_ms=50)
            st = B.scs_server_stats(srv)
        finally:
            B.scs_server_destroy(srv)
        print("server stats", st)
        assert len(done) == len(reqs) and all(d["status"] == 0 for d in done)
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["hbm_peak"] <= budget and st["max_inflight"] <= 4
        assert all(d["t_submit"] <= d["t_admit"] <= d["t_launch"] <= d["t_done"] for d in done)
        # alone: the same particles through scs_evaluate
        for q in reqs:
            B.scs_define_segmentation(q["h"], q["N"], B.SCS_SEG_EQUAL_SNR, q["G"])
            u = np.empty(q["th"].shape[0])
            B.scs_evaluate(q["h"], np.ascontiguousarray(q["th"]), u, q["prec"])
            assert np.array_equal(u, q["ups"]), (q["N"], q["th"].shape[0], q["prec"])
    finally:
        B.scs_ctx_destroy(hl)
        B.scs_ctx_destroy(hw)


def test_served_full_size_sampled():
    """The request loop on searches of the served benchmark at full size (2^20
    and 2^21 bins, G = 1024, the benchmark's segment ladder and swarm sizes,
    server shape as in `bench.py --mode serve`): every request completes and
    sampled particles of every request agree with the oracle, FP64 and
    mixed."""
    import oracle as O

    streams = synth.served_streams()
    searches = []
    for w in (streams[1], streams[2]):
        g = O.Grid(w.grid.K, w.grid.k0, w.grid.df, 2)
        m = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=w.grid.t_obs)
        psd = synth.psd_arrays(w)
        ds = D.make(g, m, psd, w.injection, w.snr, w.seed, True, w.prior_lo, w.prior_hi)
        searches.append((w, ds, _ctx(ds, w.G)))
    rng = np.random.default_rng(17)
    reqs = []
    for r in range(6):
        si = r % 2
        w, ds, h = searches[si]
        P = int(np.exp(rng.uniform(np.log(256), np.log(16384))))
        N = int(rng.choice([4096, 1024, 256, 64, 16]))
        reqs.append(dict(si=si, N=N, th=synth.particles(w.prior_lo, w.prior_hi, P, 1000 + r),
                         prec=B.SCS_PREC_MIXED if r % 3 == 2 else B.SCS_PREC_FP64))
    try:
        srv = B.scs_server_create(0, max_inflight=32, hbm_budget=64 << 30, n_streams=4)
        try:
            for q in reqs:
                q["ups"] = np.full(q["th"].shape[0], -1.0)
                B.scs_server_submit(srv, searches[q["si"]][2], q["N"], q["th"], q["ups"], q["prec"])
            done = []
            t_end = time.time() + 90
            while len(done) < len(reqs) and time.time() < t_end:
                done += B.scs_server_poll(srv, wait_ms=50)
        finally:
            B.scs_server_destroy(srv)
        assert len(done) == len(reqs) and all(d["status"] == 0 for d in done)
        worst = {B.SCS_PREC_FP64: 0.0, B.SCS_PREC_MIXED: 0.0}
        for q in reqs:
            w, ds, _ = searches[q["si"]]
            assert np.all(np.isfinite(q["ups"]))
            idx = rng.choice(q["th"].shape[0], 2, replace=False)
            r = O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, q["th"][idx], q["N"], O.SEG_EQUAL_SNR, w.G,
                           want_bounds=True)
            ref = r["ups"]
            e = PT.floored(q["ups"][idx], ref, PT.n_eff(r["bounds"]))
            worst[q["prec"]] = max(worst[q["prec"]], e.max())
            assert e.max() < (1e-9 if q["prec"] == B.SCS_PREC_FP64 else 1e-5), (q["N"], q["th"].shape[0], e)
        print(f"served at 2^20 / 2^21 bins: fp64 sampled max floored rel err {worst[B.SCS_PREC_FP64]:.3g}, "
              f"mixed {worst[B.SCS_PREC_MIXED]:.3g}")
    finally:
        for _, _, h in searches:
            B.scs_ctx_destroy(h)


def test_server_memory_stays_within_budget():
    """Admission charges the device memory the request slots actually hold
    (each keeps its buffers at the largest size it has served): requests of
    alternating shapes (many particles and few segments, then few particles
    and many segments, which grow different buffers of a slot) never make the
    server hold more than its budget, by its own count and by the device's
    free memory, and every result still equals the solo evaluation."""
    lisa = D.lisa_small(seed=23)
    h = _ctx(lisa, 16)
    try:
        shapes = [(16000, 16), (2000, 4096), (8000, 256), (3000, 1024)] * 3
        fps = [B.scs_footprint(h, P, N, B.SCS_PREC_FP64) for P, N in shapes]
        budget = int(2.5 * max(fps))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        srv = B.scs_server_create(0, max_inflight=4, hbm_budget=budget, n_streams=2)
        reqs = []
        try:
            for k, (P, N) in enumerate(shapes):
                th = D.lisa_particles(P, seed=400 + k)
                ups = np.full(P, -1.0)
                B.scs_server_submit(srv, h, N, th, ups, B.SCS_PREC_FP64)
                reqs.append((N, th, ups))
            done = []
            t_end = time.time() + 60
            while len(done) < len(reqs) and time.time() < t_end:
                done += B.scs_server_poll(srv, wait_ms=50)
            st = B.scs_server_stats(srv)
            held = free0 - torch.cuda.mem_get_info()[0]
        finally:
            B.scs_server_destroy(srv)
        print(f"budget {budget / 2**20:.1f} MiB, server count peak {st['hbm_peak'] / 2**20:.1f} MiB, "
              f"held at the end {held / 2**20:.1f} MiB")
        assert len(done) == len(reqs) and all(d["status"] == 0 for d in done)
        assert st["hbm_peak"] <= budget and st["hbm_in_use"] <= budget
        # device view: the slots' buffers, plus launch descriptors, streams and
        # allocation rounding (a few MiB against a budget of ~0.6 GB)
        assert held <= budget + (32 << 20), (held, budget)
        for N, th, ups in reqs:
            B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, 16)
            u = np.empty(th.shape[0])
            B.scs_evaluate(h, th, u)
            assert np.array_equal(u, ups), (N, th.shape[0])
    finally:
        B.scs_ctx_destroy(h)
