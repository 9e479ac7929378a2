"""Brute-force pins of the oracle's D^2 sampling (paper, Section II,
Algorithm 1: P(n_l) = d_sn(l) / sum_w d_sn(w)).

On tiny integer point sets the exact law of the ordered seed tuple is
enumerated with rational arithmetic:
    P(i_0) = 1/N,  P(i_m | i_<m) = D_m(i_m) / sum_i D_m(i),
with D_m the squared distance to the nearest of i_0..i_{m-1}.  The oracle's
draws over many Philox seeds must fit that law (chi-square), and the
inverse-CDF rule must map every interval of [0, T) to its index.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import tiny

POINTS = [
    np.array([[0, 0], [1, 0], [0, 2], [3, 3], [-2, 1], [5, -1]], dtype=np.float32),
    np.array([[0], [1], [3], [7], [8]], dtype=np.float32),
    np.array([[0, 0], [0, 0], [4, 0], [0, 3], [1, 1]], dtype=np.float32),   # a duplicate point
]


def exact_law(X, K):
    X = [tuple(int(v) for v in row) for row in X]
    N = len(X)

    def d2(a, b):
        return sum((p - q) ** 2 for p, q in zip(a, b))

    law = {}

    def rec(prefix, p):
        if len(prefix) == K:
            law[tuple(prefix)] = law.get(tuple(prefix), 0) + p
            return
        D = [min(d2(X[i], X[s]) for s in prefix) for i in range(N)]
        T = sum(D)
        for i in range(N):
            if D[i]:
                rec(prefix + [i], p * Fraction(D[i], T))

    for i0 in range(N):
        rec([i0], Fraction(1, N))
    assert sum(law.values()) == 1
    return law


def _binned(law, counts, M):
    """Observed and expected counts per tuple; tuples expected fewer than 5
    times are pooled into one bin so the chi-square approximation holds."""
    keys = sorted(law)
    obs = np.array([counts.get(k, 0) for k in keys], dtype=float)
    exp = np.array([float(law[k]) * M for k in keys])
    small = exp < 5
    if small.any():
        obs = np.append(obs[~small], obs[small].sum())
        exp = np.append(exp[~small], exp[small].sum())
    return obs, exp


@pytest.mark.parametrize("pi", range(len(POINTS)))
@pytest.mark.parametrize("K", [2, 3])
def test_tuple_frequencies_match_exact_law(oracle_lib, pi, K):
    X = POINTS[pi]
    law = exact_law(X, K)
    M = 60000
    counts = {}
    for s in range(M):
        r = oracle.seed(X, K, seed=s)
        counts[tuple(int(v) for v in r.idx)] = counts.get(tuple(int(v) for v in r.idx), 0) + 1
    assert set(counts) <= set(law), "oracle drew a tuple of probability zero"
    obs, exp = _binned(law, counts, M)
    chi2 = ((obs - exp) ** 2 / exp).sum()
    p = stats.chi2.sf(chi2, len(obs) - 1)
    assert p > 1e-4, (chi2, p)


def test_chi_square_has_power_against_a_planted_mistake():
    """Sampling proportional to the distance instead of its square (a
    plausible slip) must fail the same chi-square test."""
    X = POINTS[0]
    K = 2
    law = exact_law(X, K)
    M = 60000
    N = X.shape[0]
    counts = {}
    for s in range(M):
        u0 = tiny.uniform(s, 0)
        i0 = min(int(u0 * N), N - 1)
        D = np.sqrt(((X - X[i0]) ** 2).sum(1).astype(np.float64))      # planted: d, not d^2
        S = np.cumsum(D)
        i1 = int(np.searchsorted(S, tiny.uniform(s, 1) * S[-1], side="right"))
        counts[(i0, i1)] = counts.get((i0, i1), 0) + 1
    obs, exp = _binned(law, counts, M)
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, len(obs) - 1) < 1e-6


def test_inverse_cdf_intervals(oracle_lib):
    D = np.array([0.0, 2.0, 0.0, 0.0, 1.5, 3.0, 0.0, 0.5])
    S = np.cumsum(D)
    for b in range(len(D)):
        lo = S[b - 1] if b else 0.0
        if D[b] > 0:
            assert oracle.upper_bound(S, 0.5 * (lo + S[b])) == b      # interval midpoint
            assert oracle.upper_bound(S, lo) == b                      # left end is inside
        # t exactly at a boundary S_b belongs to the next positive interval
        nxt = next((j for j in range(b + 1, len(D)) if D[j] > 0), len(D))
        assert oracle.upper_bound(S, S[b]) == nxt
    assert oracle.upper_bound(S, 0.0) == 1      # the zero-D first point can never be drawn


def test_exhaustive_small_enumeration_matches_tiny(oracle_lib):
    """Every ordered pair of a small set reachable by the oracle's first two
    draws has the probability the exact law gives, checked on the draw rule
    itself: the oracle's second index for u in each interval."""
    X = POINTS[1]
    N = X.shape[0]
    for i0 in range(N):
        r = oracle.seed(X, 2, seed=0, replay=[i0, 0])
        D = ((X[:, 0] - X[i0, 0]) ** 2).astype(np.float64)
        S = np.cumsum(D)
        assert r.rec[1, oracle.REC_T] == S[-1]
        for i in range(N):
            if D[i] == 0:
                continue
            lo = S[i - 1] if i else 0.0
            assert oracle.upper_bound(S, 0.5 * (lo + S[i])) == i


@pytest.mark.parametrize("K", [1, 2, 3])
def test_tuple_support(oracle_lib, K):
    X = POINTS[2]
    law = exact_law(X, K)
    for s in range(2000):
        t = tuple(int(v) for v in oracle.seed(X, K, seed=s).idx)
        assert t in law
    if K >= 2:
        for t in law:
            # the duplicate pair (0,1) can never follow each other
            assert not (0 in t and 1 in t)
    assert all(len(set(t)) == len(t) for t in law)
