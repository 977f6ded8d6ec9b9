"""The launch-shape autotuners (per evaluation class and per batch) and the
request loop's admission limits.

The tuned shape changes only the order of the partial sums (chunk joins),
so tuned results agree with the default shape to rounding and with the
oracle to the FP64 bar; the cache file written by one context lets another
skip the timing.  A request whose footprint exceeds the server's HBM budget
is refused with EBUSY before any device work, and requests still waiting
when the server is destroyed are dropped without touching their buffers.
"""
import numpy as np
import pytest

import oracle as O
from tests import datasets as D
from tests import parity as PT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_13170_amd import B  # noqa: E402


def _ctx(ds, N, G=16):
    g = ds.grid
    h = B.scs_ctx_create(0)
    B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
    m = ds.model
    B.scs_set_model(h, m.pn_order, m.response, m.support, m.t_obs)
    B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, G)
    return h


def _eval(h, th, prec):
    u = torch.empty(th.shape[0], dtype=torch.float64, device="cuda")
    B.scs_evaluate(h, th, u, prec)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def test_autotune_cache_and_results(tmp_path):
    ds = D.lisa_small(seed=31)
    N, P = 64, 700
    theta = D.lisa_particles(P, seed=131)
    th = torch.tensor(np.ascontiguousarray(theta), device="cuda")
    cache = tmp_path / "tune.txt"
    h1, h2 = _ctx(ds, N), _ctx(ds, N)
    try:
        base = {p: _eval(h1, th, p) for p in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED)}
        for p in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
            B.scs_autotune(h1, th, N, p, str(cache))
        recs = [ln.split() for ln in cache.read_text().splitlines()]
        assert len(recs) == 2 and all(len(r) == 5 for r in recs), recs  # "key waves blocks L alt"
        for _, w, cb, L, alt in recs:
            assert int(w) in (1, 2, 4) and int(cb) >= 1 and int(L) in (256, 512, 1024) and int(alt) in (0, 1)
        _, bnd = B.scs_last_bounds(h1, P, N)
        for p, tol in ((B.SCS_PREC_FP64, 1e-12), (B.SCS_PREC_MIXED, 1e-5)):
            tuned = _eval(h1, th, p)
            e = PT.floored(tuned, base[p], PT.n_eff(bnd))
            print("tuned vs default shape", p, e.max())
            assert e.max() < tol
        # a second context reads the cache: a hit needs no particles at all
        lib = B.lib()
        for p in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
            assert lib.scs_autotune(h2, P, None, N, p, str(cache).encode()) == 0
        # a miss (other swarm-size class) without particles is an argument error
        assert lib.scs_autotune(h2, 8 * P, None, N, B.SCS_PREC_FP64, str(cache).encode()) == B.SCS_EINVAL
        u2 = _eval(h2, th, B.SCS_PREC_FP64)
        assert np.array_equal(u2, _eval(h1, th, B.SCS_PREC_FP64))
        ref = O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, theta[:6], N, O.SEG_EQUAL_SNR, 16, want_bounds=True)
        PT.check_rows(ds, theta[:6], u2[:6], ref, bnd[:6], 16, PT.TOL64, what="tuned vs oracle")
    finally:
        B.scs_ctx_destroy(h1)
        B.scs_ctx_destroy(h2)


def test_autotune_batch(tmp_path):
    """The batch tuner times whole batched evaluations (launch occupancy,
    then each item's LDS block and chunk); afterwards batched results agree
    with the default shapes to rounding and with the oracle, and a second
    call is answered from the cache file."""
    ds = D.lisa_small(seed=33)
    levels = [(64, 900, 133), (16, 300, 134), (1, 128, 135)]
    h = _ctx(ds, 64)
    cache = tmp_path / "tune_batch.txt"
    try:
        items, thetas = [], []
        for N, P, seed in levels:
            theta = D.lisa_particles(P, seed=seed)
            thetas.append(theta)
            items.append((h, N, torch.tensor(np.ascontiguousarray(theta), device="cuda"),
                          torch.empty(P, dtype=torch.float64, device="cuda")))

        def batched(prec):
            B.scs_evaluate_batched(items, prec)
            torch.cuda.synchronize()
            return [it[3].cpu().numpy().copy() for it in items]

        base = {p: batched(p) for p in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED)}
        for p in (B.SCS_PREC_FP64, B.SCS_PREC_MIXED):
            B.scs_autotune_batch(items, p, str(cache))
        recs = [ln.split() for ln in cache.read_text().splitlines()]
        print("batch tuner records:", recs)
        assert len(recs) == 6 and all(len(r) == 5 for r in recs)
        # N_eff per level from a solo evaluation (its edges are the batch's)
        neff = []
        for (N, P, _), it in zip(levels, items):
            B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, 16)
            B.scs_evaluate(h, it[2], torch.empty(P, dtype=torch.float64, device="cuda"))
            torch.cuda.synchronize()
            neff.append(PT.n_eff(B.scs_last_bounds(h, P, N)[1]))
        for p, tol in ((B.SCS_PREC_FP64, 1e-12), (B.SCS_PREC_MIXED, 1e-5)):
            tuned = batched(p)
            for (N, P, _), a, b, ne in zip(levels, tuned, base[p], neff):
                e = PT.floored(a, b, ne)
                print("batch-tuned vs default shapes", p, N, e.max())
                assert e.max() < tol, (p, N, e.max())
        N, P, _ = levels[0]
        B.scs_define_segmentation(h, N, B.SCS_SEG_EQUAL_SNR, 16)
        u = torch.empty(P, dtype=torch.float64, device="cuda")
        B.scs_evaluate(h, items[0][2], u)
        torch.cuda.synchronize()
        _, bnd = B.scs_last_bounds(h, P, N)
        ref = O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, thetas[0][:6], N, O.SEG_EQUAL_SNR, 16, want_bounds=True)
        PT.check_rows(ds, thetas[0][:6], batched(B.SCS_PREC_FP64)[0][:6], ref, bnd[:6], 16, PT.TOL64,
                      what="batch-tuned vs oracle")
        mtime = cache.stat().st_mtime_ns
        B.scs_autotune_batch(items, B.SCS_PREC_FP64, str(cache))  # every item cached: no timing, no rewrite
        assert cache.stat().st_mtime_ns == mtime
    finally:
        B.scs_ctx_destroy(h)


def test_server_budget_and_drop_on_destroy():
    ds = D.lisa_small(seed=32)
    h = _ctx(ds, 16)
    theta = D.lisa_particles(300, seed=132)
    srv = B.scs_server_create(0, max_inflight=1, hbm_budget=64 << 20, n_streams=1)
    try:
        big = np.tile(theta, (400, 1))  # 120000 particles: about 140 MB of workspace
        ups_big = np.full(big.shape[0], -1.0)
        with pytest.raises(B.ScsError) as ei:
            B.scs_server_submit(srv, h, 16, big, ups_big)
        assert ei.value.code == B.SCS_EBUSY and "budget" in str(ei.value)
        assert np.all(ups_big == -1.0)
        # a request that fits is served and equals the evaluation alone
        ups = np.full(300, -1.0)
        rid = B.scs_server_submit(srv, h, 16, theta, ups)
        done = []
        for _ in range(200):
            done += B.scs_server_poll(srv, wait_ms=50)
            if done:
                break
        assert [d["id"] for d in done] == [rid] and done[0]["status"] == 0
        st = B.scs_server_stats(srv)
        assert st["submitted"] == 1 and st["completed"] == 1 and st["failed"] == 0
        # the idle slot keeps its buffers for reuse, and they stay charged
        assert 0 < st["hbm_in_use"] <= st["hbm_peak"] <= 64 << 20
    finally:
        B.scs_server_destroy(srv)
    th = torch.tensor(np.ascontiguousarray(theta), device="cuda")
    alone = _eval(h, th, B.SCS_PREC_FP64)
    assert np.array_equal(ups, alone)
    # destroy with requests still queued: they are dropped, their buffers untouched
    srv = B.scs_server_create(0, max_inflight=1, hbm_budget=1 << 30, n_streams=1)
    bufs = [np.full(300, -1.0) for _ in range(6)]
    try:
        for b in bufs:
            B.scs_server_submit(srv, h, 16, theta, b)
    finally:
        B.scs_server_destroy(srv)
    served = [b for b in bufs if not np.all(b == -1.0)]
    for b in served:
        assert np.array_equal(b, alone)
    print("served before destroy:", len(served), "of", len(bufs))
    B.scs_ctx_destroy(h)


def test_launch_profile():
    """scs_ctx_profile: main launches of evaluations made while it is enabled
    are counted and timed, none while it is disabled, and enabling it again
    starts afresh (the query returns the counts before the change)."""
    ds = D.lisa_small(seed=4)
    th = torch.tensor(D.lisa_particles(64, seed=10), device="cuda")
    u = torch.empty(64, dtype=torch.float64, device="cuda")
    h = _ctx(ds, 8)
    try:
        B.scs_ctx_profile(h, 1)
        for _ in range(3):
            B.scs_evaluate(h, th, u)
        torch.cuda.synchronize()
        n, ms = B.scs_ctx_profile(h, 0)
        assert n >= 3 and n % 3 == 0 and ms > 0.0
        B.scs_evaluate(h, th, u)
        torch.cuda.synchronize()
        assert B.scs_ctx_profile(h) == (n, ms)
        assert B.scs_ctx_profile(h, 1) == (n, ms)
        assert B.scs_ctx_profile(h) == (0, 0.0)
    finally:
        B.scs_ctx_destroy(h)
