"""Plain CPU oracle of the hierarchical multi-swarm search (arXiv:2408.13170,
Sec 3.1 - 3.2 and the PSO appendix app:PSO_params).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/`` may
import it.  It shares no code with the HIP library; the PSO moves and best
updates come from this package's own ``pso_move`` / ``pso_best``, the
objective is a caller-given function (the tests pass the oracle's Upsilon_N).

The search, step by step (Sec 3.2):
  1. n_swarms swarms of equal size, positions uniform in the prior box.
  2. A rung fixes N (the objective is Upsilon_N) and the PSO hyper-parameters
     of tab:PSO_hyperparams.  Every swarm that has not converged takes PSO
     iterations: move (not on a swarm's first iteration), evaluate, bests.
  3. A swarm has converged once its best value rose by at most conv_tol over
     its last conv_window iterations (2 over 50 in app:PSO_params).  The rung
     ends when every swarm has converged or after max_iters iterations.
  4. Before every rung but the first, all particles of all swarms are
     re-grouped by k-means on their positions; every non-empty cluster becomes
     a swarm, so the number of particles is conserved.

Readings where the paper leaves the choice open (the library follows the same
ones): k of the k-means is the initial number of swarms; the positions are
clustered as features scaled to the prior box, a periodic dimension as the
point (cos, sin) / 2 pi of its angle; the k-means is k-means++ seeding
(Arthur & Vassilvitskii 2007) with draws from splitmix64 (Steele, Lea & Flood
2014) followed by Lloyd iterations until no label changes, ties going to the
lower cluster index, empty clusters dropped and clusters numbered by first
appearance; a re-grouped particle keeps its position, velocity and best
position, its best value restarts at -inf (the objective changed), and its new
swarm's best position starts at the best position of its member with the
highest earlier best value, with a swarm best value of -inf (see
``Search.regroup``); swarms are numbered in creation order, which with the
search seed keys their random numbers.
"""
from __future__ import annotations

import math

import numpy as np

from . import pso_best, pso_init, pso_move

_M64 = (1 << 64) - 1


class SplitMix64:
    """splitmix64: state += 0x9E3779B97F4A7C15, output = the state through
    two xor-shift-multiply rounds and a final xor-shift."""

    def __init__(self, seed):
        self.s = seed & _M64

    def next(self):
        self.s = (self.s + 0x9E3779B97F4A7C15) & _M64
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def uniform(self):
        """A double in (0, 1): the top 53 bits, centred in their cell."""
        return ((self.next() >> 11) + 0.5) * 2.0 ** -53


def _sqdist(x, c):
    """Squared Euclidean distance of every row of x to the point c, summed
    over the dimensions in order."""
    s = np.zeros(x.shape[0])
    for j in range(x.shape[1]):
        t = x[:, j] - c[j]
        s = s + t * t
    return s


def kmeans(x, k, iters=100, seed=0):
    """k-means of the rows of x [n, dim] into at most k clusters.
    Returns (labels [n], centres [k_out, dim])."""
    x = np.asarray(x, dtype=np.float64)
    n, dim = x.shape
    if n < 1 or dim < 1 or k < 1 or iters < 1:
        raise ValueError("bad k-means arguments")
    k = min(k, n)
    rng = SplitMix64(seed)
    # k-means++: the first centre a uniform pick, each next one a pick with
    # probability proportional to the squared distance to the nearest centre so far
    c = np.empty((k, dim))
    first = min(int(rng.uniform() * n), n - 1)
    c[0] = x[first]
    d2 = np.full(n, np.inf)
    for m in range(1, k):
        d2 = np.minimum(d2, _sqdist(x, c[m - 1]))
        tot = 0.0
        for v in d2:
            tot += v
        if tot > 0.0:
            u = rng.uniform() * tot
            pick, acc = n - 1, 0.0
            for i in range(n):
                acc += d2[i]
                if acc >= u:
                    pick = i
                    break
        else:
            pick = min(int(rng.uniform() * n), n - 1)
        c[m] = x[pick]
    # Lloyd: assign to the nearest centre (the lower index on a tie), move each
    # non-empty cluster's centre to its mean; stop when no label changes
    lab = np.full(n, -1)
    for it in range(iters):
        dist = np.stack([_sqdist(x, c[m]) for m in range(k)], axis=1)
        new = np.argmin(dist, axis=1)  # first minimum: the lower index
        changed = bool(np.any(new != lab))
        lab = new
        if not changed and it > 0:
            break
        for m in range(k):
            members = x[lab == m]
            if members.shape[0] > 0:
                s = np.zeros(dim)
                for row in members:
                    s = s + row
                c[m] = s / members.shape[0]
    # drop empty clusters, number the rest by first appearance
    order = list(dict.fromkeys(lab.tolist()))
    remap = {old: new for new, old in enumerate(order)}
    return np.array([remap[v] for v in lab.tolist()], dtype=np.int32), c[order]


def features(theta, lo, hi, periodic):
    """Clustering coordinates of positions theta [P, 7]: (theta - lo) / (hi - lo)
    per dimension, a periodic dimension as (cos, sin)(2 pi u) / 2 pi."""
    cols = []
    for d in range(theta.shape[1]):
        w = hi[d] - lo[d]
        u = (theta[:, d] - lo[d]) / w if w > 0 else np.zeros(theta.shape[0])
        if periodic[d]:
            a = 2.0 * math.pi * u
            cols += [np.cos(a) / (2.0 * math.pi), np.sin(a) / (2.0 * math.pi)]
        else:
            cols.append(u)
    return np.stack(cols, axis=1)


def converged(history, tol, window):
    """The swarm's best value rose by at most tol over its last window iterations."""
    h = len(history)
    return h > window and math.isfinite(history[h - 1 - window]) and history[-1] - history[h - 1 - window] <= tol


class Swarm:
    """A swarm's state.  Best values start at -inf; the best positions start
    at the particles' own positions, or at the positions given (a re-grouped
    swarm keeps its particles' earlier best positions as attractors)."""

    def __init__(self, theta, vel, swarm_id, pbest=None, gbest=None):
        P = theta.shape[0]
        self.theta, self.vel, self.id = theta, vel, swarm_id
        self.pbest = theta.copy() if pbest is None else pbest.copy()
        self.pbest_val = np.full(P, -np.inf)
        self.gbest = (theta[0] if gbest is None else gbest).copy()
        self.gbest_val = -np.inf
        self.iteration = 0


class Search:
    """The search state across rungs.  objective(theta [P, 7], N) -> values [P]
    (NaN for an invalid position)."""

    def __init__(self, objective, n_swarms, particles, lo, hi, periodic, seed, conv_tol=2.0, conv_window=50,
                 kmeans_iters=100):
        self.objective = objective
        self.lo, self.hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
        self.periodic = np.asarray(periodic, dtype=np.int32)
        self.seed, self.k = seed, n_swarms
        self.conv_tol, self.conv_window, self.kmeans_iters = conv_tol, conv_window, kmeans_iters
        self.next_id = 0
        self.rungs_done = 0
        self.swarms = []
        for _ in range(n_swarms):
            th = pso_init(particles, self.lo, self.hi, seed, self.next_id)
            self.swarms.append(Swarm(th, np.zeros_like(th), self.next_id))
            self.next_id += 1

    def regroup(self):
        """k-means on all positions (Sec 3.2); every cluster becomes a swarm.
        Positions, velocities and best positions carry over; best values
        restart at -inf because the objective changed.  Positions outside the
        prior box score -inf, so a best position is always inside the box:
        keeping them as attractors pulls a cluster of particles that stand
        outside the box back in.  The swarm's best position starts at the
        best position of its particle with the highest earlier best value
        (the first such particle on ties)."""
        th = np.concatenate([s.theta for s in self.swarms])
        vel = np.concatenate([s.vel for s in self.swarms])
        pb = np.concatenate([s.pbest for s in self.swarms])
        pv = np.concatenate([s.pbest_val for s in self.swarms])
        f = features(th, self.lo, self.hi, self.periodic)
        lab, _ = kmeans(f, self.k, self.kmeans_iters, self.seed ^ (0x6B6D65616E73 + self.rungs_done))
        self.swarms = []
        for c in range(int(lab.max()) + 1):
            sel = lab == c
            j = int(np.argmax(pv[sel]))
            self.swarms.append(Swarm(th[sel].copy(), vel[sel].copy(), self.next_id, pbest=pb[sel], gbest=pb[sel][j]))
            self.next_id += 1

    def step(self, sw, N, prm):
        omega, phi_p, phi_g, eps = prm
        if sw.iteration > 0:
            pso_move(sw.theta, sw.vel, sw.pbest, sw.gbest, omega, phi_p, phi_g, eps, self.lo, self.hi, self.periodic,
                     self.seed, sw.id, sw.iteration)
        vals = self.objective(sw.theta, N)
        sw.gbest_val = pso_best(sw.theta, vals, self.lo, self.hi, self.periodic, sw.pbest, sw.pbest_val, sw.gbest,
                                sw.gbest_val)
        sw.iteration += 1

    def run_rung(self, N, max_iters, prm):
        """One rung; prm = (Omega, Phi_P, Phi_G, eps[7]).  Returns the report."""
        if self.rungs_done > 0:
            self.regroup()
        n = len(self.swarms)
        hist = [[] for _ in range(n)]
        done = [False] * n
        it = 0
        while it < max_iters:
            active = [i for i in range(n) if not done[i]]
            if not active:
                break
            for i in active:
                self.step(self.swarms[i], N, prm)
                hist[i].append(self.swarms[i].gbest_val)
                done[i] = converged(hist[i], self.conv_tol, self.conv_window)
            it += 1
            if all(done):
                break
        self.rungs_done += 1
        return {"N": N, "n_swarms": n, "iterations": it, "converged": int(sum(done)),
                "best_val": max((h[-1] for h in hist if h), default=-np.inf)}

    def bests(self):
        """Per swarm: (size, best position [7], best value)."""
        return [(s.theta.shape[0], s.gbest.copy(), s.gbest_val) for s in self.swarms]
