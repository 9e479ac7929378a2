"""Pins for the oracle's k-means|| (Bahmani et al., "Scalable K-Means++",
PVLDB 2012, Algorithm 2; the different initialisation the paper's
introduction attributes to Bahmani et al.).

* D before a round: torch.cdist (library) squared distance to the first
  point; phi: math.fsum within the recursive-summation bound;
* inclusion law: over many Philox seeds the number of times each point joins
  in round 1 matches the sum of min(1, ell * D / phi) (Bernoulli sums, z
  test per point and over all points);
* weights: nearest-candidate counts from torch.cdist (ties to the smaller
  candidate index), summing to N;
* weighted recluster: the law of the first two centres by exact rational
  enumeration (first proportional to w, second to w * D^2) on a fixed
  candidate set, chi-square over seeds;
* special cases: huge ell takes every point with D > 0 in round 1, zero
  rounds keep only the first point, identical points never join and warn;
* a well-separated mixture: every component holds a centre in nearly all
  runs and the cost stays within a small factor of k-means++.
"""
import math
from fractions import Fraction

import numpy as np
import torch

import kmpp_synth
import oracle


def _d2(X, C):
    return torch.cdist(torch.from_numpy(X).double(), torch.from_numpy(C).double()).square().numpy()


def test_first_round_distances_and_phi(oracle_lib):
    X = kmpp_synth.gaussian(3000, 5, seed=11).numpy()
    r = oracle.kmpar(X, 8, seed=4, rounds=2, keep_D=True)
    D0 = _d2(X, X[r.cand[:1]])[:, 0]
    np.testing.assert_allclose(r.Dr[0], D0, rtol=1e-12, atol=0)
    assert abs(r.phi[0] - math.fsum(r.Dr[0])) <= 3000 * 2.0 ** -53 * r.phi[0]
    # D before round 2: nearest of the candidates that joined so far
    D1 = _d2(X, X[r.cand[:r.round_end[1]]]).min(axis=1)
    np.testing.assert_allclose(r.Dr[1], D1, rtol=1e-12, atol=0)


def test_inclusion_law_over_seeds(oracle_lib):
    # 12 integer points; count how often each joins in round 1 against the
    # sum of its inclusion probabilities (which depend on the random first
    # point) over 4000 seeds
    X = np.array([[0, 0], [1, 0], [0, 2], [3, 1], [5, 5], [6, 5], [9, 0], [9, 1], [2, 7], [4, 4], [8, 8], [1, 9]],
                 np.float32)
    N, ell = X.shape[0], 3.0
    hits = np.zeros(N)
    psum, pvar = np.zeros(N), np.zeros(N)
    bsum, bvar = np.zeros(N), np.zeros(N)   # a planted mistake: D instead of D^2
    for s in range(4000):
        r = oracle.kmpar(X, 2, seed=s, rounds=1, ell=ell, keep_D=True)
        p = np.minimum(1.0, ell * r.Dr[0] / r.phi[0])
        psum += p
        pvar += p * (1 - p)
        q = np.sqrt(r.Dr[0])
        b = np.minimum(1.0, ell * q / q.sum())
        bsum += b
        bvar += b * (1 - b)
        hits[r.cand[r.round_end[0]:r.round_end[1]]] += 1
    z = (hits - psum) / np.sqrt(np.maximum(pvar, 1e-12))
    assert np.all(np.abs(z) < 5), z
    assert abs(hits.sum() - psum.sum()) / math.sqrt(pvar.sum()) < 5
    zb = (hits - bsum) / np.sqrt(np.maximum(bvar, 1e-12))
    assert np.max(np.abs(zb)) > 5


def test_weights_are_nearest_candidate_counts(oracle_lib):
    X = kmpp_synth.lattice(5000, 3, lim=6, seed=2).numpy()   # many exact ties
    r = oracle.kmpar(X, 6, seed=9, rounds=3)
    d2 = _d2(X, X[r.cand])
    nearest = d2.argmin(axis=1)                            # first minimum: smallest index
    np.testing.assert_array_equal(r.labels, nearest)
    np.testing.assert_array_equal(r.weights, np.bincount(nearest, minlength=r.ncand))
    assert r.weights.sum() == 5000


def test_weighted_recluster_law_by_enumeration(oracle_lib):
    # fixed candidates and weights (replayed), K = 2: P(first = a) = w_a / W,
    # P(second = b | a) = w_b D(b, a) / sum_c w_c D(c, a)
    X = np.array([[0, 0], [4, 0], [0, 3], [10, 10], [1, 1]], np.float32)
    cand = np.array([0, 1, 2, 3])
    w = np.array([5, 1, 2, 3])
    end = np.array([1, 4])
    pts = X[cand].astype(np.int64)
    law = {}
    for a in range(4):
        pa = Fraction(int(w[a]), int(w.sum()))
        dd = [int(((pts[b] - pts[a]) ** 2).sum()) for b in range(4)]
        tot = sum(int(w[b]) * dd[b] for b in range(4))
        for b in range(4):
            if dd[b]:
                law[(a, b)] = pa * Fraction(int(w[b]) * dd[b], tot)
    M = 30000
    counts = {}
    for s in range(M):
        r = oracle.kmpar(X, 2, seed=s, rounds=1, ell=1.0, replay_cand=cand, replay_end=end, replay_w=w)
        key = (int(np.nonzero(cand == r.idx[0])[0][0]), int(np.nonzero(cand == r.idx[1])[0][0]))
        counts[key] = counts.get(key, 0) + 1
    assert set(counts) <= set(law)
    chi2 = sum((counts.get(k, 0) - M * float(p)) ** 2 / (M * float(p)) for k, p in law.items())
    # 12 cells, 11 degrees of freedom: the 1e-4 upper quantile is about 38
    assert chi2 < 38, chi2


def test_special_cases(oracle_lib):
    X = kmpp_synth.gaussian(500, 4, seed=3).numpy()
    # huge ell: every point with D > 0 joins in round 1
    r = oracle.kmpar(X, 5, seed=1, rounds=1, ell=1e15)
    assert r.ncand == 500 and sorted(r.cand[1:].tolist()) == [i for i in range(500) if i != r.cand[0]]
    assert np.all(r.weights == 1)
    # zero rounds: the first point alone, holding every point
    r = oracle.kmpar(X, 1, seed=2, rounds=0)
    assert r.ncand == 1 and r.weights.tolist() == [500] and r.idx.tolist() == r.cand.tolist()
    assert r.cand[0] == min(int(math.floor(oracle.uniform(2, 0) * 500)), 499)
    # identical points: phi = 0, nobody joins; K = 2 needs a uniform draw
    Z = np.ones((50, 3), np.float32)
    r = oracle.kmpar(Z, 2, seed=5, rounds=3)
    assert r.ncand == 1 and r.status == oracle.W_DEGENERATE


def test_separated_mixture_quality(oracle_lib):
    rng = np.random.default_rng(5)
    g = np.stack(np.meshgrid(np.arange(4), np.arange(4)), -1).reshape(-1, 2) * 1000.0
    z = rng.permutation(np.repeat(np.arange(16), 300))
    X = (g[z] + rng.standard_normal((4800, 2))).astype(np.float32)
    hit_all, cost_par, cost_pp = 0, [], []
    for s in range(40):
        r = oracle.kmpar(X, 16, seed=s, rounds=5)
        hit_all += len(set(z[r.idx].tolist())) == 16
        cost_par.append(_d2(X, X[r.idx]).min(axis=1).sum())
        cost_pp.append(oracle.seed(X, 16, seed=s).phi)
    assert hit_all >= 38
    assert np.mean(cost_par) <= 2.0 * np.mean(cost_pp)
