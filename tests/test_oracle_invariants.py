"""Invariants, closed forms and special cases that pin the FP64 oracle
(paper, Section II, Algorithms 1 and 2).

* D is the nearest-seed squared distance: it never increases from one step
  to the next, is zero at every chosen seed, and equals min over seeds of
  torch.cdist in FP64 (a library routine);
* the prefix total is within the recursive-summation error bound of
  math.fsum of D (the correctly rounded sum);
* scaling X by a power of two, or translating an integer lattice by an
  integer vector, leaves every draw unchanged (exact metamorphic tests);
* the incremental C oracle and the recompute-all NumPy oracle agree;
* expected cost identities: with one uniform seed E[phi] = 2 * sum ||x-mean||^2
  exactly (Arthur & Vassilvitskii, Lemma 3.1), and for K=2 the exact E[phi]
  from enumeration matches the Monte-Carlo mean of the oracle;
* on a well-separated mixture the mean cost over 1000 seeds is within
  statistical error of 2 * sum of within-cluster SSE, and below the
  8 (ln K + 2) phi_OPT bound;
* special cases: K=1, N=K, two points, all points equal, a NaN row.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import tiny
import kmpp_synth


def _gauss(N, d, seed, scale=1.0):
    return kmpp_synth.gaussian(N, d, seed=seed, scale=scale).numpy()


def _D_after(X, idx_prefix):
    """D after the passes for the given seeds, via replay (K = len)."""
    K = len(idx_prefix)
    return oracle.seed(X, K, replay=idx_prefix).D


@pytest.mark.parametrize("N,d,K,seed", [(200, 2, 8, 0), (333, 5, 12, 3), (64, 17, 20, 9)])
def test_c_oracle_matches_recompute_all(oracle_lib, N, d, K, seed):
    X = _gauss(N, d, seed)
    r = oracle.seed(X, K, seed=seed)
    idx, D = tiny.seed(X.astype(np.float32), K, seed=seed)
    assert list(r.idx) == idx
    np.testing.assert_allclose(r.D, D, rtol=1e-12, atol=0)
    rz = oracle.seed(X, K, seed=seed, zero_seed_rows=True)
    idz, Dz = tiny.seed(X.astype(np.float32), K, seed=seed, zero_seed_rows=True)
    assert list(rz.idx) == idz
    np.testing.assert_allclose(rz.D, Dz, rtol=1e-12, atol=0)


def test_D_monotone_zero_at_seeds_and_cdist(oracle_lib):
    X = _gauss(500, 6, 1)
    K = 25
    r = oracle.seed(X, K, seed=5)
    prev = None
    prevT = math.inf
    for m in range(1, K + 1):
        D = _D_after(X, list(r.idx[:m]))
        C = torch.from_numpy(X[r.idx[:m]]).double()
        ref = torch.cdist(torch.from_numpy(X).double(), C).square().min(dim=1).values.numpy()
        np.testing.assert_allclose(D, ref, rtol=1e-10, atol=1e-12)
        assert np.all(D[r.idx[:m]] == 0.0)
        if prev is not None:
            assert np.all(D <= prev)
        prev = D
        if m < K:
            T = r.rec[m, oracle.REC_T]
            # recursive FP64 summation of non-negative terms: relative error
            # at most (N-1) * 2^-53 (Higham, Accuracy and Stability of
            # Numerical Algorithms, section 4.2)
            assert T == pytest.approx(math.fsum(D), rel=(len(D) - 1) * 2.0 ** -53, abs=0)
            assert T <= prevT
            prevT = T
    assert len(set(r.idx.tolist())) == K


def test_power_of_two_scaling_is_exact(oracle_lib):
    X = _gauss(700, 4, 2)
    a = oracle.seed(X, 30, seed=11)
    b = oracle.seed(X * 8.0, 30, seed=11)
    c = oracle.seed(X * 0.25, 30, seed=11)
    assert list(a.idx) == list(b.idx) == list(c.idx)
    np.testing.assert_array_equal(a.D * 64.0, b.D)


def test_integer_translation_is_exact(oracle_lib):
    X = kmpp_synth.lattice(400, 3, seed=1).numpy()
    shift = np.array([17.0, -9.0, 40.0], dtype=np.float32)
    a = oracle.seed(X, 40, seed=2)
    b = oracle.seed(X + shift, 40, seed=2)
    assert list(a.idx) == list(b.idx)
    np.testing.assert_array_equal(a.D, b.D)


def test_one_uniform_seed_expected_cost_identity(oracle_lib):
    X = _gauss(300, 3, 4, scale=2.0)
    N = X.shape[0]
    phis = [oracle.seed(X, 1, replay=[i]).phi for i in range(N)]
    Xd = X.astype(np.float64)
    sse = ((Xd - Xd.mean(axis=0)) ** 2).sum()
    assert np.mean(phis) == pytest.approx(2.0 * sse, rel=1e-12)


def test_two_seed_expected_cost_enumeration_vs_monte_carlo(oracle_lib):
    X = _gauss(40, 2, 6)
    N = X.shape[0]
    exact = 0.0
    for i0 in range(N):
        D1 = _D_after(X, [i0])
        p1 = D1 / D1.sum()
        for i1 in range(N):
            if p1[i1] > 0:
                exact += p1[i1] / N * oracle.seed(X, 2, replay=[i0, i1]).phi
    M = 20000
    phis = np.array([oracle.seed(X, 2, seed=s).phi for s in range(M)])
    se = phis.std() / math.sqrt(M)
    assert abs(phis.mean() - exact) < 4 * se


def test_expected_cost_on_well_separated_mixture(oracle_lib):
    # 16 means on a 4x4 grid at spacing 1000, sigma 1, d 2, 625 points each
    K, n, d = 16, 625, 2
    g = torch.Generator().manual_seed(77)
    grid = torch.stack(torch.meshgrid(torch.arange(4.0), torch.arange(4.0), indexing="ij"), -1).reshape(K, d)
    means = grid.double() * 1000.0
    lab = torch.arange(K).repeat_interleave(n)
    X = (means[lab] + torch.randn((K * n, d), generator=g, dtype=torch.float64)).float().numpy()
    Xd = X.astype(np.float64)
    sse = 0.0
    for j in range(K):
        P = Xd[lab.numpy() == j]
        sse += ((P - P.mean(0)) ** 2).sum()
    M = 1000
    phis = np.array([oracle.seed(X, K, seed=s).phi for s in range(M)])
    target = 2.0 * sse
    rel_sd = 1.0 / math.sqrt(2 * d * K)           # per-run relative spread
    assert abs(phis.mean() / target - 1.0) < 4 * rel_sd / math.sqrt(M) + 2e-3
    assert phis.mean() <= 8.0 * (math.log(K) + 2.0) * sse


def test_special_K1(oracle_lib):
    X = _gauss(123, 3, 8)
    r = oracle.seed(X, 1, seed=42)
    i0 = min(int(math.floor(oracle.uniform(42, 0) * 123)), 122)
    assert list(r.idx) == [i0]
    ref = ((X.astype(np.float64) - X[i0].astype(np.float64)) ** 2).sum(1)
    np.testing.assert_allclose(r.D, ref, rtol=1e-14)
    lab, _, _ = oracle.assign(X, X[r.idx])
    assert np.all(lab == 0)


def test_special_N_equals_K(oracle_lib):
    X = _gauss(50, 4, 9)
    r = oracle.seed(X, 50, seed=3)
    assert sorted(r.idx.tolist()) == list(range(50))
    assert np.all(r.D == 0.0)
    lab, _, _ = oracle.assign(X, X[r.idx])
    inv = np.empty(50, dtype=np.int64)
    inv[r.idx] = np.arange(50)
    np.testing.assert_array_equal(lab, inv)


def test_special_two_points(oracle_lib):
    X = np.array([[1.0, 2.0], [4.0, -2.0]], dtype=np.float32)
    for s in range(20):
        r = oracle.seed(X, 2, seed=s)
        assert r.idx[1] == 1 - r.idx[0]
        assert r.status == oracle.OK


def test_special_all_identical_is_degenerate(oracle_lib):
    X = np.ones((30, 3), dtype=np.float32)
    r = oracle.seed(X, 4, seed=1)
    assert r.status == oracle.W_DEGENERATE
    for m in range(1, 4):
        assert r.idx[m] == min(int(math.floor(oracle.uniform(1, m) * 30)), 29)


def test_special_nan_row_is_nonfinite(oracle_lib):
    X = _gauss(30, 3, 10)
    X[7, 1] = np.nan
    r = oracle.seed(X, 3, seed=0)
    assert r.status == oracle.E_NONFINITE


def test_replay_acceptance_rule():
    # own index i=3 with interval [10, 12); t = 10.000001 is near the boundary 10
    rec = np.zeros(8)
    rec[oracle.REC_T] = 100.0
    rec[oracle.REC_t] = 10.00000005
    rec[oracle.REC_SI_LO], rec[oracle.REC_SI_HI] = 10.0, 12.0
    rec[oracle.REC_SG_LO], rec[oracle.REC_SG_HI], rec[oracle.REC_DG] = 9.0, 10.0, 1.0
    assert oracle.seed_index_ok(3, rec, own=3)
    assert oracle.seed_index_ok(2, rec, own=3)          # neighbour across a near boundary
    rec[oracle.REC_t] = 11.0                             # far from any boundary
    assert not oracle.seed_index_ok(2, rec, own=3)
