"""Pins of the oracle's single draw with u given (paper, Section II,
Algorithm 1: the next seed is point l with probability d_sn(l) / sum_w
d_sn(w), read as the inverse CDF in index order): the first index whose
inclusive FP64 prefix exceeds t = u * sum(D), the boundary rule (t equal to
a prefix value goes to the next positive interval), the rounding fallback
(no prefix exceeds t: the last index with D > 0), the degenerate and
non-finite cases, and the same rule in the weighted recluster of k-means||.

Every D here is a small integer (or a dyadic fraction), so every prefix sum
and every t used is exact in FP64 and the expected index follows from the
definition with integer arithmetic, independently of the oracle's code.
The replay in ranges is pinned to the whole run, bit for bit."""
import numpy as np
import pytest

import oracle


def first_above(D, t):
    """Definition: the first i with sum(D[:i+1]) > t (exact integer sums)."""
    s = 0
    for i, v in enumerate(D):
        s += v
        if s > t:
            return i
    return None


def test_boundaries_and_fallback_by_hand():
    D = [0, 1, 0, 2, 1, 0, 0]          # S = 0 1 1 3 4 4 4, T = 4
    cases = {0.0: 1,                    # t = 0: the first positive D
             0.125: 1,                  # t = 0.5 inside (0, 1)
             0.25: 3,                   # t = 1 = S_1 = S_2: the next positive interval
             0.5: 3,                    # t = 2 inside (1, 3)
             0.75: 4,                   # t = 3 = S_3
             0.96875: 4,                # t = 3.875
             1.0: 4}                    # t = T: no prefix exceeds it -> last D > 0 (not N-1)
    for u, want in cases.items():
        i, st, rec = oracle.draw(np.array(D, float), u)
        assert st == oracle.OK
        assert i == want, (u, i, want)
        T, t, lo, hi = rec
        assert T == 4.0 and t == 4.0 * u
        assert hi == sum(D[:i + 1]) and lo == sum(D[:i])
        if u < 1.0:
            assert lo <= t < hi


def test_fallback_skips_trailing_zeros_and_single_positive():
    # u = 1 is outside the stream's range [0, 1); it is the only way to make
    # t reach the total exactly, which is what rounding can do on the GPU
    for D, want in [([0, 0, 5, 0, 0, 0], 2), ([3, 0, 0], 0), ([0, 0, 0, 7], 3), ([1, 1, 1, 1], 3)]:
        i, st, _ = oracle.draw(np.array(D, float), 1.0)
        assert st == oracle.OK and i == want, (D, i)


def test_degenerate_and_nonfinite():
    i, st, rec = oracle.draw(np.zeros(7), 0.5)
    assert st == oracle.W_DEGENERATE and i == 3          # floor(0.5 * 7)
    i, st, _ = oracle.draw(np.zeros(7), 0.9999999)
    assert st == oracle.W_DEGENERATE and i == 6
    for bad in (np.nan, np.inf):
        D = np.ones(5)
        D[2] = bad
        i, st, _ = oracle.draw(D, 0.3)
        assert st == oracle.E_NONFINITE and i == -1


@pytest.mark.parametrize("N", [9, 1000, 200_003])
def test_every_boundary_and_midpoint_against_the_definition(N):
    # integer D (zeros included) across several 65,536-row prefix chunks:
    # every prefix is an exact integer, T is a power of two after scaling u
    rng = np.random.default_rng(N)
    D = rng.integers(0, 4, N).astype(np.int64)
    D[rng.random(N) < 0.3] = 0
    T = int(D.sum())
    S = np.cumsum(D)
    # t at every boundary S_b and midway inside intervals (a sample for big N)
    marks = np.unique(S)[:-1]
    if marks.size > 300:
        marks = np.concatenate([marks[:100], rng.choice(marks, 100, replace=False), marks[-100:]])
    Df = D.astype(float)
    for b in marks:
        for t in (float(b), float(b) + 0.5):
            u = t / T                       # u * T may round; use the t the oracle forms
            i, st, rec = oracle.draw(Df, u)
            assert st == oracle.OK
            tt = rec[1]
            assert tt == np.float64(u) * np.float64(T)
            want = int(np.searchsorted(S, tt, side="right"))
            assert want < N
            assert i == want, (t, i, want)
            assert D[i] > 0


def test_weighted_recluster_draw():
    share = [0, 2, 0, 0, 3, 0]         # S = 0 2 2 2 5 5, T = 5
    for u, want in {0.0: 1, 0.2: 1, 0.4: 4, 0.9: 4, 1.0: 4}.items():
        j, st, rec = oracle.wdraw(np.array(share, float), u)
        assert st == oracle.OK and j == want, (u, j)
        assert j == (first_above(share, rec[1]) if u < 1.0 else 4)
    j, st, _ = oracle.wdraw(np.zeros(4), 0.6)
    assert st == oracle.W_DEGENERATE and j == 2
    j, st, _ = oracle.wdraw(np.array([1.0, np.inf]), 0.1)
    assert st == oracle.E_NONFINITE


@pytest.mark.parametrize("zero_rows,replay", [(False, False), (True, False), (False, True)])
def test_range_replay_equals_whole_run(zero_rows, replay):
    rng = np.random.default_rng(5)
    X = rng.normal(size=(3_001, 5)).astype(np.float32)
    K = 23
    base = oracle.seed(X, K, seed=7, zero_seed_rows=zero_rows)
    rp = None
    if replay:   # a different but valid seed sequence
        rp = np.roll(base.idx, 3)
        rp[0] = base.idx[0]
        base = oracle.seed(X, K, seed=7, zero_seed_rows=zero_rows, replay=rp)
    seen = []
    r = oracle.seed(X, K, seed=7, zero_seed_rows=zero_rows, replay=rp, chunk=6, progress=seen.append)
    assert seen == [6, 12, 18, 23]
    assert np.array_equal(r.idx, base.idx)
    assert np.array_equal(r.D, base.D)
    assert np.array_equal(r.rec, base.rec)
    assert r.status == base.status
