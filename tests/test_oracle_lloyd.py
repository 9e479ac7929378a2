"""Pins for the oracle's Lloyd iterations (after seeding the clustering
proceeds as standard k-means, paper Section II): one iteration assigns every
point to its nearest centre and moves every centre to the mean of its
points; an empty cluster keeps its centre.

* hand-worked iterations (tests/golden/lloyd_hand.txt);
* the update against a library group mean (numpy add.at in FP64);
* K = 1 closed form: the centre is the mean and the second cost is the
  total sum of squares about it;
* well-separated mixture: from k-means++ seeds Lloyd reaches the component
  sample means and the cost equals the sum of the components' SSE;
* invariants: cost never increases; at convergence the state is a fixed
  point (centres are the means, every point nearest its own centre).
"""
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    rows = []
    with open(os.path.join(HERE, "golden", "lloyd_hand.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = [c.strip() for c in line.split("|")]
            d = int(p[1])
            rows.append(dict(case=int(p[0]), d=d, X=np.array(p[2].split(), float).reshape(-1, d),
                             C0=np.array(p[3].split(), float).reshape(-1, d), it=int(p[4]),
                             labels=np.array(p[5].split(), int), cost=float(p[6]), changed=int(p[7]),
                             C=np.array(p[8].split(), float).reshape(-1, d)))
    return rows


@pytest.mark.parametrize("row", _golden(), ids=lambda r: f"case{r['case']}-it{r['it']}")
def test_hand_worked_iterations(oracle_lib, row):
    C, lab, cost, ch = oracle.lloyd(row["X"], row["C0"], row["it"])
    np.testing.assert_array_equal(lab, row["labels"])
    assert cost[-1] == pytest.approx(row["cost"], rel=1e-6)
    assert int(ch[-1]) == row["changed"]
    np.testing.assert_array_equal(C, row["C"].astype(np.float32))


def test_update_is_the_group_mean(oracle_lib):
    rng = np.random.default_rng(0)
    N, d, K = 5000, 7, 40
    X = (rng.standard_normal((N, d)) * 10).astype(np.float32)
    lab = rng.integers(0, K - 1, N).astype(np.int32)    # cluster K-1 left empty
    C_prev = rng.standard_normal((K, d)).astype(np.float32)
    C, n = oracle.lloyd_update(X, lab, C_prev)
    s = np.zeros((K, d))
    np.add.at(s, lab, X.astype(np.float64))
    cnt = np.bincount(lab, minlength=K)
    np.testing.assert_array_equal(n, cnt)
    ref = np.where(cnt[:, None] > 0, s / np.maximum(cnt, 1)[:, None], C_prev.astype(np.float64)).astype(np.float32)
    # summation order differs from add.at only by FP64 rounding: the FP32
    # results agree to one unit in the last place
    np.testing.assert_array_max_ulp(C, ref, maxulp=1)
    np.testing.assert_array_equal(C[K - 1], C_prev[K - 1])


def test_single_cluster_closed_form(oracle_lib):
    rng = np.random.default_rng(1)
    X = (rng.standard_normal((3000, 5)) * 3 + 7).astype(np.float32)
    c0 = X[17:18]
    C, lab, cost, ch = oracle.lloyd(X, c0, 2)
    xd = X.astype(np.float64)
    mean = xd.mean(axis=0).astype(np.float32)
    np.testing.assert_array_max_ulp(C[0], mean, maxulp=1)
    assert cost[0] == pytest.approx(((xd - c0.astype(np.float64)) ** 2).sum(), rel=1e-12)
    assert cost[1] == pytest.approx(((xd - C[0].astype(np.float64)) ** 2).sum(), rel=1e-12)
    # the cost about the FP32-rounded mean exceeds the exact minimum only by
    # N * ||mean - x_bar||^2
    sse = ((xd - xd.mean(axis=0)) ** 2).sum()
    assert sse <= cost[1] <= sse * (1 + 1e-9)
    assert list(ch) == [3000, 0] and np.all(lab == 0)


def _separated(seed):
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(np.arange(4), np.arange(4)), -1).reshape(-1, 2) * 1000.0
    z = rng.permutation(np.repeat(np.arange(16), 625))
    X = (g[z] + rng.standard_normal((10000, 2))).astype(np.float32)
    return X, z


def test_separated_mixture_reaches_component_means(oracle_lib):
    X, z = _separated(5)
    r = oracle.seed(X, 16, seed=3)
    assert len(set(z[r.idx].tolist())) == 16          # one seed per component
    C, lab, cost, ch = oracle.lloyd(X, X[r.idx], 3)
    xd = X.astype(np.float64)
    means = np.stack([xd[z == k].mean(axis=0) for k in range(16)])
    comp = z[r.idx]                                    # component of each seed
    np.testing.assert_array_max_ulp(C, means[comp].astype(np.float32), maxulp=1)
    np.testing.assert_array_equal(comp[lab], z)        # partition = the components
    sse = sum(((xd[z == k] - means[k]) ** 2).sum() for k in range(16))
    assert cost[2] == pytest.approx(sse, rel=1e-6)
    assert list(ch[1:]) == [0, 0]


def test_cost_never_increases_and_ends_at_a_fixed_point(oracle_lib):
    rng = np.random.default_rng(7)
    means = rng.uniform(-5, 5, (12, 3))
    X = (means[rng.integers(0, 12, 4000)] + rng.standard_normal((4000, 3))).astype(np.float32)
    r = oracle.seed(X, 12, seed=1)
    C, lab, cost, ch = oracle.lloyd(X, X[r.idx], 200)
    assert np.all(np.diff(cost) <= 1e-12 * cost[:-1])
    assert ch[-1] == 0
    # fixed point: centres are the means of their points, each point nearest
    # its own centre
    C2, _ = oracle.lloyd_update(X, lab, C)
    np.testing.assert_array_equal(C2, C)
    l2, _, _ = oracle.assign(X, C)
    np.testing.assert_array_equal(l2, lab)
