"""GPU parity of the Lloyd iterations after seeding (paper, Section II: the
clustering proceeds as standard k-means once the centroids are chosen)
against the FP64 oracle, through the C ABI.

Replay: each iteration is checked on the GPU's own previous centres, so one
legitimate near-tie difference cannot cascade:
  * labels equal to the oracle's nearest centre, or the GPU's centre within
    1e-5 relative of the oracle's nearest distance (near tie);
  * new centres against the oracle's FP64 means of the GPU's labels, within
    one FP32 unit in the last place plus the fixed-point rounding bound
    max|x| * 2^(ceil(log2 N) - 61);
  * cost (FP64 sum of the direct FP32 distances) within 1e-5 relative of the
    oracle's FP64 cost; changed-label counts and cluster sizes exact.
Integer lattices: the first update is bit-exact.
"""
import math

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


def check_labels(Xd, C, lab_gpu):
    ol, om, _ = oracle.assign(Xd, C)
    bad = np.nonzero(lab_gpu != ol)[0]
    if bad.size:
        dg = oracle.pair_dist(Xd, bad, C, lab_gpu[bad])
        assert np.all(dg - om[bad] <= 1e-5 * om[bad]), "labels differ beyond the near-tie rule"
    return om


def check_centres(C_gpu, C_or, Xd):
    amax = float(np.abs(Xd).max())
    lgN = math.ceil(math.log2(max(2, Xd.shape[0])))
    tol = np.spacing(np.abs(C_or).astype(np.float32)).astype(np.float64) + amax * 2.0 ** (lgN - 61)
    err = np.abs(C_gpu.astype(np.float64) - C_or.astype(np.float64))
    assert np.all(err <= tol), f"worst centre error {float(err.max()):.3e}"


def replay(kl, X, Xd, C0, iters, **kw):
    """Run `iters` single iterations on the GPU and check each one."""
    C = C0.clone()
    N = X.shape[0]
    prev = None
    for t in range(iters):
        C_before = C.cpu().numpy().copy()
        C, lab, cost, ch, counts, ws = kl.kmpp_lloyd(X, C, 1, **kw)
        assert kl.kmpp_status(ws) == 0
        torch.cuda.synchronize()
        lab_h = lab.cpu().numpy()
        om = check_labels(Xd, C_before, lab_h)
        C_or, n_or = oracle.lloyd_update(Xd, lab_h, C_before)
        check_centres(C.cpu().numpy(), C_or, Xd)
        np.testing.assert_array_equal(counts.cpu().numpy(), n_or)
        assert int(ch[0]) == N
        dsel = oracle.pair_dist(Xd, np.arange(N), C_before, lab_h)
        assert float(cost[0]) == pytest.approx(float(dsel.sum()), rel=1e-5)
        assert float(cost[0]) >= float(om.sum()) * (1 - 1e-5)
        prev = lab_h
    return C, prev


def test_lloyd_small_workload_replay(kl):
    w = kmpp_synth.small()
    X = w.X.cuda()
    _say("small N=10000 d=2 K=16")
    idx, C0, _, _ = kl.kmpp_seed(X, w.K, 0)
    C_step, lab_step = replay(kl, X, w.X.numpy(), C0, 8)
    # one call of 8 iterations: the same centres and labels, bit for bit
    C, lab, cost, ch, counts, _ = kl.kmpp_lloyd(X, C0.clone(), 8)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(C.cpu().numpy(), C_step.cpu().numpy())
    np.testing.assert_array_equal(lab.cpu().numpy(), lab_step)
    c = cost.cpu().numpy()
    assert np.all(np.diff(c) <= 1e-6 * c[:-1]), c
    chh = ch.cpu().numpy()
    assert chh[0] == w.N and np.all(chh[1:] <= w.N)


@pytest.mark.parametrize("d", [1, 2, 3, 8])
def test_lloyd_lattice_first_update_bit_exact(kl, d):
    N, K = 40_003, 25
    Xh = kmpp_synth.lattice(N, d, seed=20 + d)
    X = Xh.cuda()
    _say("lattice", N, d, K)
    C0 = X[torch.arange(0, N, N // K, device="cuda")[:K]].contiguous()
    C, lab, cost, ch, counts, _ = kl.kmpp_lloyd(X, C0.clone(), 1)
    torch.cuda.synchronize()
    C_or, lab_or, cost_or, ch_or = oracle.lloyd(Xh.numpy(), C0.cpu().numpy(), 1)
    np.testing.assert_array_equal(lab.cpu().numpy(), lab_or)
    np.testing.assert_array_equal(C.cpu().numpy(), C_or)
    assert float(cost[0]) == float(cost_or[0])
    assert int(ch[0]) == int(ch_or[0]) == N


@pytest.mark.parametrize("d,K", [(5, 40), (17, 300), (64, 256), (100, 20), (300, 9),
                                 (128, 1024), (33, 2000), (512, 100), (64, 1000)])
def test_lloyd_shapes_and_paths(kl, d, K):
    # the cluster sums of one LDS range hold about 47 KiB: up to 3 ranges the
    # LDS path, from 4 ranges on (the last four shapes) the sorted path
    N = 30_011
    Xh = kmpp_synth.gaussian(N, d, seed=700 + d)
    X = Xh.cuda()
    _say("gaussian", N, d, K)
    idx, C0, _, _ = kl.kmpp_seed(X, K, 1)
    replay(kl, X, Xh.numpy(), C0, 3)


def test_lloyd_plain_workload(kl):
    w = kmpp_synth.plain(device="cuda")
    _say("plain N=1000000 d=32 K=256, 3 iterations")
    idx, C0, _, _ = kl.kmpp_seed(w.X, w.K, 0)
    replay(kl, w.X, w.X.cpu().numpy(), C0, 3)


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_lloyd_precision_forms(kl, fmt):
    N, d, K = 100_003, 128, 64
    Xh = kmpp_synth.gaussian(N, d, seed=800, scale=3.0)
    X = Xh.cuda()
    dt = kl.DTYPES[fmt]
    Xq, E = kl.kmpp_quantize(X, dt)
    if fmt == "bf16":
        Xd = oracle.bf16_decode(oracle.bf16_encode(Xh.numpy()))
    else:
        Xd = oracle.fp8_dequantize_rows(*oracle.fp8_quantize_rows_fast(Xh.numpy()))
    _say(fmt, N, d, K)
    idx, C0, _, _ = kl.kmpp_seed(X, K, 2, Xq=Xq, Xq_exp=E, dtype=dt)
    replay(kl, Xq, Xd, C0, 3, X_exp=E, dtype=dt)


@pytest.mark.parametrize("fmt,d,K", [("bf16", 128, 300), ("bf16", 100, 400), ("bf16", 129, 300),
                                     ("fp8", 256, 200), ("fp8", 130, 300), ("fp8", 64, 600)])
def test_lloyd_precision_forms_sorted_path(kl, fmt, d, K):
    # K * d large enough for the sorted path (at least four cluster ranges),
    # BF16 and FP8 rows of even, odd and ragged widths
    N = 30_011
    Xh = kmpp_synth.gaussian(N, d, seed=900 + d, scale=3.0)
    X = Xh.cuda()
    dt = kl.DTYPES[fmt]
    Xq, E = kl.kmpp_quantize(X, dt)
    if fmt == "bf16":
        Xd = oracle.bf16_decode(oracle.bf16_encode(Xh.numpy()))
    else:
        Xd = oracle.fp8_dequantize_rows(*oracle.fp8_quantize_rows_fast(Xh.numpy()))
    _say(fmt, "sorted path", N, d, K)
    idx, C0, _, _ = kl.kmpp_seed(X, K, 3, Xq=Xq, Xq_exp=E, dtype=dt)
    replay(kl, Xq, Xd, C0, 2, X_exp=E, dtype=dt)


def test_lloyd_sorted_path_determinism(kl):
    # the sorted path's scatter order varies from run to run; the integer
    # sums do not, so two runs give the same bits
    N, d, K = 50_021, 128, 1024
    Xh = kmpp_synth.gaussian(N, d, seed=901)
    X = Xh.cuda()
    idx, C0, _, _ = kl.kmpp_seed(X, K, 2)
    _say("sorted path determinism", N, d, K)
    outs = [kl.kmpp_lloyd(X, C0.clone(), 3) for _ in range(2)]
    torch.cuda.synchronize()
    for a, b in zip(outs[0][:5], outs[1][:5]):
        assert torch.equal(a, b)


def test_lloyd_determinism_and_empty_clusters(kl):
    N, d, K = 50_000, 4, 12
    Xh = kmpp_synth.gaussian(N, d, seed=900)
    X = Xh.cuda()
    C0 = torch.cat([X[:10], torch.full((2, d), 1e4, device="cuda")]).contiguous()  # two far centres stay empty
    _say("determinism / empty clusters")
    outs = [kl.kmpp_lloyd(X, C0.clone(), 5) for _ in range(2)]
    torch.cuda.synchronize()
    np.testing.assert_array_equal(outs[0][0].cpu().numpy(), outs[1][0].cpu().numpy())
    np.testing.assert_array_equal(outs[0][2].cpu().numpy(), outs[1][2].cpu().numpy())
    C = outs[0][0].cpu().numpy()
    np.testing.assert_array_equal(C[10:], np.full((2, d), 1e4, np.float32))
    assert np.all(outs[0][4].cpu().numpy()[10:] == 0)
    C_or, lab_or, cost_or, ch_or = oracle.lloyd(Xh.numpy(), C0.cpu().numpy(), 5)
    check_centres(C, C_or, Xh.numpy())


def test_lloyd_edge_cases(kl):
    Xh = kmpp_synth.gaussian(1000, 6, seed=901)
    X = Xh.cuda()
    # K = 1: the mean of all rows after one iteration, then nothing changes
    C, lab, cost, ch, counts, _ = kl.kmpp_lloyd(X, X[3:4].clone(), 2)
    torch.cuda.synchronize()
    mean = Xh.numpy().astype(np.float64).mean(axis=0)
    check_centres(C.cpu().numpy()[0], mean.astype(np.float32), Xh.numpy())
    assert ch.cpu().tolist() == [1000, 0] and int(counts[0]) == 1000
    # N = K: every row its own centre
    C, lab, cost, ch, counts, _ = kl.kmpp_lloyd(X[:20].contiguous(), X[:20].clone(), 1)
    torch.cuda.synchronize()
    assert lab.cpu().tolist() == list(range(20)) and float(cost[0]) == 0.0
    np.testing.assert_array_equal(C.cpu().numpy(), Xh.numpy()[:20])
    # zero iterations leave the centres alone
    C0 = X[:5].clone()
    C, *_ = kl.kmpp_lloyd(X, C0, 0)
    np.testing.assert_array_equal(C.cpu().numpy(), Xh.numpy()[:5])
    # non-finite input
    Xn = X.clone()
    Xn[7, 2] = float("nan")
    *_, ws = kl.kmpp_lloyd(Xn, X[:4].clone(), 1)
    assert kl.kmpp_status(ws) == -4
    with pytest.raises(kl.KmppError):
        kl.kmpp_lloyd(X, X[:4].clone(), -1)
