"""The hierarchical multi-swarm search (Sec 3.1 - 3.2, app:PSO_params) on the
20000-bin A+E case: a three-rung ladder with the rung hyper-parameters of
tab:PSO_hyperparams (minimum speeds scaled to the narrow test box), k-means
re-grouping between rungs, the convergence rule, particle conservation,
determinism, that the final coherent rung sits on the injected peak, and
rung-by-rung agreement with the search oracle."""
import numpy as np
import pytest

import oracle as O
import synth
from tests import datasets as D
from tests import parity as PT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_13170_amd import B  # noqa: E402

# (N, Omega, Phi_P, Phi_G, eps): the rows of tab:PSO_hyperparams for N = 100, 10
# and 1, with the minimum speeds divided by 10 for a box ~10x narrower than the
# paper's prior (order of theta: Mc, eta, f_low, lambda, beta, iota, psi)
LADDER = [(16, 0.5, 0.2, 0.3, [0.01, 0.005, 5e-9, 0.01, 0.01, 0.02, 0.01]),
          (4, 0.3, 0.2, 0.5, [0.0001, 0.005, 1e-9, 0.0001, 0.0001, 0.001, 0.01]),
          (1, 0.72, 1.193, 1.193, [0.0] * 7)]


def _ctx(ds):
    g = ds.grid
    h = B.scs_ctx_create(0)
    B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(ds.psd), g.k0 * g.df, g.df)
    m = ds.model
    B.scs_set_model(h, m.pn_order, m.response, m.support, m.t_obs)
    B.scs_define_segmentation(h, 1, B.SCS_SEG_EQUAL_SNR, 16)
    return h


def _search(h, inj, seed):
    lo = inj - np.array([0.15, 0.02, 2e-6, 0.15, 0.15, 0.3, 0.3])
    hi = inj + np.array([0.15, 0.02, 2e-6, 0.15, 0.15, 0.3, 0.3])
    hi[1] = min(hi[1], 0.25)
    s = B.scs_search_create(h, 3, 256, lo, hi, synth.PERIODIC, G=16, conv_tol=2.0, conv_window=8, kmeans_iters=50,
                            seed=seed)
    reports, sizes = [], []
    try:
        for N, om, pp, pg, eps in LADDER:
            rep = B.scs_search_run_rung(s, N, 30, B.pso_params(om, pp, pg, eps))
            sz, best = B.scs_search_swarms(s)
            reports.append(rep)
            sizes.append(sz)
            print(rep, "sizes", list(sz), "bests", np.round(best[:, 7], 2))
        return reports, sizes, best
    finally:
        B.scs_search_destroy(s)


def test_search_ladder():
    ds = D.lisa_small(seed=27)
    h = _ctx(ds)
    try:
        inj = ds.injection
        u = torch.empty(1, dtype=torch.float64, device="cuda")
        B.scs_evaluate(h, torch.tensor(inj[None, :], device="cuda"), u)
        torch.cuda.synchronize()
        ups_inj = float(u[0])
        reports, sizes, best = _search(h, inj, seed=5)
        for (N, *_), rep, sz in zip(LADDER, reports, sizes):
            assert rep["N"] == N and 1 <= rep["iterations"] <= 30
            assert 0 <= rep["converged"] <= rep["n_swarms"] == len(sz)
            assert sz.sum() == 3 * 256 and np.all(sz > 0)
        # the coherent rung ends on the injected peak
        top = int(np.argmax(best[:, 7]))
        print("best Upsilon_1", best[top, 7], "at the injection", ups_inj)
        assert best[top, 7] >= 0.98 * ups_inj
        # the reported best is Upsilon_1 of that position (evaluated alone, bit for bit)
        B.scs_define_segmentation(h, 1, B.SCS_SEG_EQUAL_SNR, 16)
        B.scs_evaluate(h, torch.tensor(best[top:top + 1, :7], device="cuda"), u)
        torch.cuda.synchronize()
        assert float(u[0]) == best[top, 7]
        # same seed, same search
        _, _, best2 = _search(h, inj, seed=5)
        assert np.array_equal(best, best2)
        # a window longer than the rung: nothing converges, every iteration runs
        w = np.array([0.01, 0.002, 1e-6, 0.01, 0.01, 0.01, 0.01])
        s = B.scs_search_create(h, 2, 64, inj - w, inj + w, synth.PERIODIC, conv_window=1000, seed=1)
        try:
            rep = B.scs_search_run_rung(s, 8, 4, B.pso_params(*LADDER[0][1:]))
            assert rep["iterations"] == 4 and rep["converged"] == 0 and rep["n_swarms"] == 2
            with pytest.raises(B.ScsError):
                B.scs_search_run_rung(s, 0, 4, B.pso_params(*LADDER[0][1:]))
        finally:
            B.scs_search_destroy(s)
    finally:
        B.scs_ctx_destroy(h)


def test_search_matches_oracle():
    """The library's search against the oracle's (oracle/search.py over the
    oracle's Upsilon_N), rung by rung: the same iterations, convergence and
    re-grouping (swarm sizes), the same best positions bit for bit (the PSO
    arithmetic is exact; the statistic differs by rounding only, far below
    any gap between the values compared), best values within 1e-9."""
    from oracle import search as OS

    ds = D.lisa_small(seed=31)
    inj = ds.injection
    w = np.array([0.15, 0.02, 2e-6, 0.15, 0.15, 0.3, 0.3])
    lo, hi = inj - w, inj + w
    hi[1] = min(hi[1], 0.25)
    n_sw, per, G, seed = 3, 48, 16, 123
    ladder = [(16, LADDER[0][1:]), (4, LADDER[1][1:]), (1, LADDER[2][1:])]

    def ups(th, N):
        return O.evaluate(ds.grid, ds.model, ds.d_ri, ds.psd, th, N, O.SEG_EQUAL_SNR, G)["ups"]

    ref = OS.Search(ups, n_sw, per, lo, hi, synth.PERIODIC, seed, conv_tol=2.0, conv_window=4, kmeans_iters=50)
    h = _ctx(ds)
    try:
        s = B.scs_search_create(h, n_sw, per, lo, hi, synth.PERIODIC, G=G, conv_tol=2.0, conv_window=4,
                                kmeans_iters=50, seed=seed)
        try:
            for N, (om, pp, pg, eps) in ladder:
                rep = B.scs_search_run_rung(s, N, 10, B.pso_params(om, pp, pg, eps))
                want = ref.run_rung(N, 10, (om, pp, pg, eps))
                sizes, best = B.scs_search_swarms(s)
                wb = ref.bests()
                print(f"N={N}: library {rep['iterations']} iterations, {rep['converged']} converged, sizes "
                      f"{list(sizes)}; oracle {want['iterations']}, {want['converged']}, {[b[0] for b in wb]}")
                for key in ("N", "n_swarms", "iterations", "converged"):
                    assert rep[key] == want[key], (N, key)
                assert abs(rep["best_val"] - want["best_val"]) <= 1e-9 * abs(want["best_val"])
                assert list(sizes) == [b[0] for b in wb]
                for i, (_, pos, val) in enumerate(wb):
                    assert np.array_equal(best[i, :7], pos), (N, i)
                    assert abs(best[i, 7] - val) <= 1e-9 * abs(val), (N, i, best[i, 7], val)
        finally:
            B.scs_search_destroy(s)
    finally:
        B.scs_ctx_destroy(h)


# the rows of tab:PSO_hyperparams at the paper's prior (N = 100, 50, 10, 1)
LADDER_PAPER = [(100, 0.5, 0.2, 0.3, [0.1, 0.05, 5e-8, 0.1, 0.1, 0.2, 0.1]),
                (50, 0.5, 0.2, 0.4, [0.01, 0.05, 1e-8, 0.01, 0.01, 0.2, 0.1]),
                (10, 0.3, 0.2, 0.5, [0.001, 0.05, 1e-8, 0.001, 0.001, 0.01, 0.1]),
                (1, 0.72, 1.193, 1.193, [0.0] * 7)]


def test_search_full_size_sampled():
    """The search `bench.py --mode search` runs, at full size (6 swarms x 10^4
    particles, 2^20 bins, G = 1024, the ladder N = 100, 50, 10, 1 with its
    rung hyper-parameters), cut to 4 iterations per rung: particles are
    conserved through every k-means re-grouping, every swarm's best position
    lies in the prior box and its best value equals the oracle's Upsilon_N
    there."""
    w = synth.workload("lisa1m")
    g = O.Grid(w.grid.K, w.grid.k0, w.grid.df, 2)
    m = O.Model(pn_order=7, response=O.RESP_LISA_LF_AE, support=O.SUPPORT_TOBS, t_obs=w.grid.t_obs)
    psd = synth.psd_arrays(w)
    ds = D.make(g, m, psd, w.injection, w.snr, w.seed, True, w.prior_lo, w.prior_hi)
    h = B.scs_ctx_create(0)
    try:
        B.scs_load_data(h, np.ascontiguousarray(ds.d_ri), np.ascontiguousarray(psd), g.k0 * g.df, g.df)
        B.scs_set_model(h, 7, m.response, m.support, m.t_obs)
        B.scs_define_segmentation(h, 1, B.SCS_SEG_EQUAL_SNR, w.G)
        s = B.scs_search_create(h, 6, 10000, w.prior_lo, w.prior_hi, synth.PERIODIC, G=w.G, conv_tol=2.0,
                                conv_window=50, kmeans_iters=100, seed=synth.BASE_SEED + 61)
        try:
            worst = 0.0
            for N, om, pp, pg, eps in LADDER_PAPER:
                rep = B.scs_search_run_rung(s, N, 4, B.pso_params(om, pp, pg, eps))
                sizes, best = B.scs_search_swarms(s)
                assert rep["N"] == N and 1 <= rep["iterations"] <= 4
                assert sizes.sum() == 6 * 10000 and np.all(sizes > 0)
                # best positions lie in the prior box, also for swarms re-grouped from
                # particles that stood outside it
                assert np.all((best[:, :7] >= w.prior_lo) & (best[:, :7] <= w.prior_hi))
                r = O.evaluate(g, m, ds.d_ri, psd, np.ascontiguousarray(best[:, :7]), N, O.SEG_EQUAL_SNR,
                               w.G, want_bounds=True)
                ref = r["ups"]
                e = PT.floored(best[:, 7], ref, PT.n_eff(r["bounds"]))
                worst = max(worst, e.max())
                print(f"rung N={N}: {len(sizes)} swarms {list(sizes)}, bests {np.round(best[:, 7], 2)}")
                assert e.max() < 1e-9, (N, e)
            print(f"full-size search: swarm bests against the oracle, max floored rel err {worst:.3g}")
        finally:
            B.scs_search_destroy(s)
    finally:
        B.scs_ctx_destroy(h)
