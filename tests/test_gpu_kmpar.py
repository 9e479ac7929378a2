"""GPU parity of the k-means|| initialisation (Bahmani et al., PVLDB 2012,
Algorithm 2) against the FP64 oracle, through the C ABI.

Replay: every round is checked on the D the GPU's own earlier candidates
define.  A point's join decision must equal the oracle's unless its uniform
u lies within 1e-5 * p of its probability p (FP32 distances against FP64);
labels follow the near-tie rule (1e-5); weights equal the counts of the
GPU's labels; recluster draws equal the oracle's draw from the GPU's
earlier centres and weights, or lie within 1e-6 * total of a CDF boundary.
Integer lattices make every distance and sum exact: everything must match
bit for bit.
"""
import numpy as np
import pytest
import torch

import kmpp_synth
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_02136_amd as k
    k.lib()
    return k


def _say(*a):
    print(*a, flush=True)


def _run(kl, X, K, seed, rounds, ell, **kw):
    idx, C, cand, rend, w, lab, ws = kl.kmpp_seed_parallel(X, K, seed, rounds=rounds, ell=ell, **kw)
    st = kl.kmpp_status(ws)
    torch.cuda.synchronize()
    rend = rend.cpu().numpy().astype(np.int64)
    m = int(rend[-1])
    return (idx.cpu().numpy(), C.cpu().numpy(), cand.cpu().numpy()[:m], rend, w.cpu().numpy()[:m],
            lab.cpu().numpy(), st)


def check_replay(Xh, K, seed, rounds, ell, gpu, inst=0):
    idx, C, cand, rend, w, lab, st = gpu
    N = Xh.shape[0]
    assert st >= 0, st
    np.testing.assert_array_equal(C, Xh[idx])
    r = oracle.kmpar(Xh, K, seed=seed, rounds=rounds, ell=ell, inst=inst, keep_D=True, replay_cand=cand,
                     replay_end=rend, replay_w=w, replay_idx=idx)
    assert int(r.cand[0]) == int(cand[0]), "first point"
    differ = 0
    for q in range(rounds):
        mine = set(cand[rend[q]:rend[q + 1]].tolist())
        own = set(r.cand[r.round_end[q]:r.round_end[q + 1]].tolist())
        for i in mine ^ own:
            p = min(1.0, ell * r.Dr[q][i] / r.phi[q])
            u = oracle.uniform4(seed, int(i), inst, q + 1, 1)
            assert abs(u - p) <= 1e-5 * p + 1e-12, (q, i, u, p, i in mine)
            differ += 1
        # the GPU's list keeps point order within a round
        assert np.all(np.diff(cand[rend[q]:rend[q + 1]]) > 0)
    # labels: near-tie rule against the GPU's candidate list
    bad = np.nonzero(lab != r.labels)[0]
    if bad.size:
        dg = oracle.pair_dist(Xh, bad, Xh[cand], lab[bad])
        dm = oracle.pair_dist(Xh, bad, Xh[cand], r.labels[bad])
        assert np.all(dg - dm <= 1e-5 * dm), "labels beyond the near-tie rule"
    np.testing.assert_array_equal(w, np.bincount(lab, minlength=cand.size))
    for k in range(K):
        assert oracle.seed_index_ok(int(idx[k]), r.rec[k], int(r.idx[k])), (k, int(idx[k]), int(r.idx[k]))
    return differ


@pytest.mark.parametrize("d", [1, 2, 3, 8])
def test_kmpar_lattice_bit_exact(kl, d):
    N, K, rounds = 30_011, 12, 4
    Xh = kmpp_synth.lattice(N, d, seed=40 + d)
    _say("kmpar lattice", N, d, K)
    idx, C, cand, rend, w, lab, st = _run(kl, Xh.cuda(), K, 7, rounds, 2.0 * K)
    r = oracle.kmpar(Xh.numpy(), K, seed=7, rounds=rounds, ell=2.0 * K)
    assert st == r.status
    np.testing.assert_array_equal(rend, r.round_end)
    np.testing.assert_array_equal(cand, r.cand)
    np.testing.assert_array_equal(w, r.weights)
    np.testing.assert_array_equal(lab, r.labels)
    np.testing.assert_array_equal(idx, r.idx)


@pytest.mark.parametrize("d", [2, 5, 16, 32, 64, 100, 128, 129])
def test_kmpar_gaussian_replay(kl, d):
    N, K, rounds = 40_009, 20, 5
    Xh = kmpp_synth.gaussian(N, d, seed=60 + d, scale=2.0)
    _say("kmpar gaussian", N, d, K)
    gpu = _run(kl, Xh.cuda(), K, 3, rounds, 2.0 * K)
    check_replay(Xh.numpy(), K, 3, rounds, 2.0 * K, gpu)


def test_kmpar_paper_shape_and_determinism(kl):
    w = kmpp_synth.paper_shape("paper_k")
    _say("kmpar paper shape", w.N, w.d, w.K)
    X = w.X.cuda()
    a = _run(kl, X, w.K, 0, 5, 2.0 * w.K)
    b = _run(kl, X, w.K, 0, 5, 2.0 * w.K)
    for u, v in zip(a[:6], b[:6]):
        np.testing.assert_array_equal(u, v)
    check_replay(w.X.numpy(), w.K, 0, 5, 2.0 * w.K, a)


def test_kmpar_plain_workload(kl):
    w = kmpp_synth.plain(device="cuda")
    _say("kmpar plain", w.N, w.d, w.K)
    gpu = _run(kl, w.X, w.K, 0, 5, 2.0 * w.K)
    check_replay(w.X.cpu().numpy(), w.K, 0, 5, 2.0 * w.K, gpu)


def test_kmpar_edge_cases(kl):
    Xh = kmpp_synth.gaussian(2000, 6, seed=5)
    X = Xh.cuda()
    # no rounds: the first point alone, weight N
    idx, C, cand, rend, w, lab, st = _run(kl, X, 1, 4, 0, 8.0)
    assert st == 0 and cand.size == 1 and w.tolist() == [2000] and idx.tolist() == cand.tolist()
    assert int(cand[0]) == min(int(np.floor(oracle.uniform(4, 0) * 2000)), 1999)
    # identical points: nobody joins; K = 3 draws need the uniform fallback
    Z = torch.ones((500, 4), device="cuda")
    idx, C, cand, rend, w, lab, st = _run(kl, Z, 3, 1, 3, 6.0)
    assert st == 1 and cand.size == 1
    # another instance id changes the draws
    a = _run(kl, X, 8, 2, 3, 16.0)
    b = _run(kl, X, 8, 2, 3, 16.0, instance=5)
    assert not np.array_equal(a[2], b[2])
    check_replay(Xh.numpy(), 8, 2, 3, 16.0, b, inst=5)
    # argument errors
    with pytest.raises(kl.KmppError):
        kl.kmpp_seed_parallel(X, 4, 0, ell=0.0)
    with pytest.raises(kl.KmppError):
        kl.kmpp_seed_parallel(X, 4, 0, rounds=-1)


def test_kmpar_wide_rows(kl):
    # rows beyond the matrix-core widths take the assignment's direct form
    Xh = kmpp_synth.gaussian(6_007, 300, seed=77)
    _say("kmpar wide", 6007, 300, 10)
    gpu = _run(kl, Xh.cuda(), 10, 1, 4, 20.0)
    check_replay(Xh.numpy(), 10, 1, 4, 20.0, gpu)
