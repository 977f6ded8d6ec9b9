"""Pins of the search oracle (oracle/search.py) against what fixes it from
outside: the published splitmix64 outputs, scikit-learn's k-means on
unambiguous clusters, hand-made convergence histories, and a search on a
synthetic objective whose peak is known."""
import math

import numpy as np
import pytest

from oracle import search as S


def test_splitmix64_published_outputs():
    # the first three outputs of splitmix64 from state 0 (Steele, Lea & Flood 2014)
    g = S.SplitMix64(0)
    assert [g.next() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = S.SplitMix64(0).uniform()
    assert u == ((0xE220A8397B1DCDAF >> 11) + 0.5) / 2.0 ** 53 and 0.0 < u < 1.0


def _blobs(seed, k=5, per=300, dim=7):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, (k, dim))
    while min(np.linalg.norm(a - b) for i, a in enumerate(centres) for b in centres[i + 1:]) < 0.3:
        centres = rng.uniform(0.0, 1.0, (k, dim))
    return np.concatenate([c + 0.01 * rng.standard_normal((per, dim)) for c in centres]), np.repeat(np.arange(k), per)


def test_kmeans_against_sklearn():
    cluster = pytest.importorskip("sklearn.cluster")
    metrics = pytest.importorskip("sklearn.metrics")
    x, truth = _blobs(2)
    lab, ctr = S.kmeans(x, 5, 100, seed=9)
    assert metrics.adjusted_rand_score(truth, lab) == 1.0
    ref = cluster.KMeans(n_clusters=5, n_init=10, random_state=0).fit(x)
    assert metrics.adjusted_rand_score(ref.labels_, lab) == 1.0
    for c in range(5):
        assert np.allclose(ctr[c], x[lab == c].mean(axis=0), rtol=0, atol=1e-12)
    assert list(dict.fromkeys(lab.tolist())) == list(range(5))
    # a fixed point of Lloyd: every point is nearest to its own centre
    d = np.stack([((x - c) ** 2).sum(axis=1) for c in ctr], axis=1)
    assert np.array_equal(np.argmin(d, axis=1), lab)


def test_kmeans_degenerate_inputs():
    pts = np.repeat(np.array([[0.0, 0.0], [1.0, 1.0], [0.0, 5.0]]), 4, axis=0)
    lab, ctr = S.kmeans(pts, 6, seed=1)  # more clusters than distinct points: empties dropped
    assert len(ctr) == 3 and sorted(set(lab.tolist())) == [0, 1, 2]
    for c in range(3):
        assert np.all(pts[lab == c] == pts[lab == c][0])
    lab1, ctr1 = S.kmeans(pts, 1, seed=3)  # k = 1: the mean
    assert np.all(lab1 == 0) and np.allclose(ctr1[0], pts.mean(axis=0))
    with pytest.raises(ValueError):
        S.kmeans(pts, 0)


def test_features_periodic_and_scaled():
    lo, hi = np.array([0.0, 10.0]), np.array([2.0, 20.0])
    th = np.array([[0.0, 10.0], [2.0, 15.0], [1.0, 20.0]])
    f = S.features(th, lo, hi, [1, 0])
    assert f.shape == (3, 3)
    # both ends of a periodic dimension are one point; the middle is opposite
    assert np.allclose(f[0, :2], f[1, :2], atol=1e-15)
    assert np.allclose(f[2, :2], -f[0, :2])
    assert np.allclose(np.hypot(f[:, 0], f[:, 1]), 1.0 / (2.0 * math.pi))
    assert np.allclose(f[:, 2], [0.0, 0.5, 1.0])


def test_convergence_rule():
    assert not S.converged([1.0, 2.0, 3.0], 2.0, 3)  # history not longer than the window
    assert S.converged([1.0, 2.0, 2.5, 3.0], 2.0, 3)  # gain 2 over 3 iterations: converged
    assert not S.converged([1.0, 2.0, 2.5, 3.0 + 1e-9], 2.0, 3)
    assert not S.converged([-np.inf, 5.0, 5.0, 5.0], 2.0, 3)  # no finite best a window ago
    assert S.converged([7.0, 7.0], 0.0, 1)


def test_search_on_a_known_peak():
    """A concave objective with its maximum 100 at theta0: the ladder ends
    there, particles are conserved, the report matches the rule."""
    lo = np.array([0.0, 0.0, 0.0, 0.0, -1.0, 0.0, -1.0])
    hi = np.array([1.0, 1.0, 1.0, 2 * math.pi, 1.0, math.pi, 0.0])
    theta0 = np.array([0.3, 0.6, 0.45, 2.0, 0.2, 1.5, -0.4])
    per = [0, 0, 0, 1, 0, 0, 1]
    calls = []

    def objective(th, N):
        calls.append(N)
        return 100.0 - N * np.sum(((th - theta0) / (hi - lo)) ** 2, axis=1) * 50.0

    s = S.Search(objective, 3, 40, lo, hi, per, seed=77, conv_tol=0.5, conv_window=5, kmeans_iters=50)
    reports = []
    for N, prm in ((4, (0.5, 0.2, 0.3, [0.01] * 7)), (2, (0.3, 0.2, 0.5, [0.001] * 7)),
                   (1, (0.72, 1.193, 1.193, [0.0] * 7))):
        reports.append(s.run_rung(N, 60, prm))
        assert sum(b[0] for b in s.bests()) == 120
    for r in reports:
        assert 1 <= r["iterations"] <= 60 and 0 <= r["converged"] <= r["n_swarms"] <= 3
    best = max(s.bests(), key=lambda b: b[2])
    assert best[2] > 99.0 and np.all(np.abs(best[1] - theta0) / (hi - lo) < 0.03)
    assert best[2] == pytest.approx(objective(best[1][None, :], 1)[0], abs=0)
    assert set(calls) == {4, 2, 1}
    # same seed, same search
    s2 = S.Search(objective, 3, 40, lo, hi, per, seed=77, conv_tol=0.5, conv_window=5, kmeans_iters=50)
    for N, prm in ((4, (0.5, 0.2, 0.3, [0.01] * 7)),):
        assert s2.run_rung(N, 60, prm) == reports[0]


def test_regroup_keeps_best_positions_and_restarts_values():
    """Between rungs (Sec 3.2): positions, velocities and best positions carry
    over, best values restart at -inf, and a new swarm's best position is the
    best position of its particle with the highest earlier best value.  A
    cluster of particles standing outside the prior box keeps attractors
    inside it, and its next move heads back in."""
    lo, hi = np.zeros(7), np.ones(7)
    per = np.zeros(7, dtype=np.int32)
    s = S.Search(lambda th, N: np.zeros(th.shape[0]), 2, 40, lo, hi, per, seed=3, kmeans_iters=50)
    rng = np.random.default_rng(0)
    for sw in s.swarms:
        sw.pbest = sw.theta.copy()
        sw.pbest_val = rng.normal(size=sw.theta.shape[0])
    # swarm 1's particles all stand outside the box in dimension 0
    s.swarms[1].theta[:, 0] = 1.5 + 0.01 * np.arange(40)
    th = np.concatenate([w.theta for w in s.swarms])
    pb = np.concatenate([w.pbest for w in s.swarms])
    pv = np.concatenate([w.pbest_val for w in s.swarms])
    s.rungs_done = 1
    s.regroup()
    assert sum(w.theta.shape[0] for w in s.swarms) == 80
    for w in s.swarms:
        rows = [int(np.flatnonzero(np.all(th == x, axis=1))[0]) for x in w.theta]
        assert np.array_equal(w.pbest, pb[rows])
        assert np.all(w.pbest_val == -np.inf) and w.gbest_val == -np.inf
        assert np.array_equal(w.gbest, pb[rows][int(np.argmax(pv[rows]))])
        assert np.all((w.pbest >= lo) & (w.pbest <= hi)) and np.all((w.gbest >= lo) & (w.gbest <= hi))
    outside = [w for w in s.swarms if np.all(w.theta[:, 0] > 1.0)]
    assert outside, "the out-of-box particles form a cluster of their own"
    w = outside[0]
    before = w.theta[:, 0].copy()
    S.pso_move(w.theta, w.vel, w.pbest, w.gbest, 0.5, 0.5, 0.5, np.zeros(7), lo, hi, per, 3, w.id, 1)
    assert np.all(w.theta[:, 0] < before)
