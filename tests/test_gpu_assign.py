"""GPU parity of the nearest-seed assignment (output O of the paper's
Algorithm 1) against the FP64 oracle, through the C ABI.

Bar: labels equal the oracle's, except at near-ties where the GPU's centre
is within 1e-5 relative of the oracle's nearest distance (FP64 distances);
the returned distance within 2e-5 relative of the FP64 distance to the
returned centre (FP32 direct form over d <= 300 terms)."""
import numpy as np
import pytest
import torch

import kmpp_synth
import oracle

pytestmark = pytest.mark.gpu

LABEL_RTOL = 1e-5
MIND_RTOL = 2e-5


@pytest.fixture(scope="module")
def kl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_02136_amd as k
    k.lib()
    return k


def check_assign(Xd, C, lab, mind):
    lo, mo, _ = oracle.assign(Xd, C)
    bad = np.nonzero(lab != lo)[0]
    if bad.size:
        dg = oracle.pair_dist(Xd, bad, C, lab[bad])
        worst = np.max((dg - mo[bad]) / np.maximum(mo[bad], 1e-300))
        assert np.all(dg - mo[bad] <= LABEL_RTOL * mo[bad]), f"{bad.size} labels differ, worst rel gap {worst:.2e}"
    dsel = oracle.pair_dist(Xd, np.arange(Xd.shape[0]), C, lab)
    err = np.abs(mind.astype(np.float64) - dsel)
    assert np.all(err <= MIND_RTOL * dsel + 1e-30), f"mind worst rel {np.max(err / np.maximum(dsel, 1e-30)):.2e}"
    return bad.size


def run_assign(kl, X, C, **kw):
    lab, mind, ws = kl.kmpp_assign(X, C, **kw)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), mind.cpu().numpy()


@pytest.mark.parametrize("d", [1, 2, 3, 8, 16, 32, 33, 64, 100, 128, 129, 300])
@pytest.mark.parametrize("K", [1, 17, 256])
def test_f32_shapes(kl, d, K):
    N = 5_003
    Xh = kmpp_synth.gaussian(N, d, seed=d, scale=3.0)
    Ch = Xh[torch.randperm(N, generator=torch.Generator().manual_seed(K))[:K]].contiguous()
    print("assign f32", N, d, K, flush=True)
    lab, mind = run_assign(kl, Xh.cuda(), Ch.cuda())
    check_assign(Xh.numpy(), Ch.numpy(), lab, mind)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("K", [1024, 1025])
def test_centre_setup_paths(kl, dtype, K):
    # d = 64 pads to 64 columns in both formats: K = 1024 is a centre block of
    # exactly 65,536 padded elements (prepared by one workgroup), K = 1025
    # pads to 1040 rows (the three-kernel setup)
    N, d = 3_001, 64
    Xh = kmpp_synth.gaussian(N, d, seed=K + 7 * dtype, scale=2.0)
    Ch = Xh[torch.randperm(N, generator=torch.Generator().manual_seed(K))[:K]].contiguous()
    print("assign setup path", dtype, N, d, K, flush=True)
    if dtype == 0:
        lab, mind = run_assign(kl, Xh.cuda(), Ch.cuda())
        Xd = Xh.numpy()
    else:
        q, _ = kl.kmpp_quantize(Xh.cuda(), kl.KMPP_BF16)
        lab, mind = run_assign(kl, q, Ch.cuda(), dtype=kl.KMPP_BF16)
        Xd = oracle.bf16_decode(oracle.bf16_encode(Xh.numpy()))
    check_assign(Xd, Ch.numpy(), lab, mind)


def test_exact_ties_go_to_smallest_index(kl):
    # integer lattice with duplicated centres: exact ties everywhere
    Xh = kmpp_synth.lattice(20_000, 4, lim=5, seed=1)
    Ch = torch.cat([Xh[:40], Xh[:40], Xh[10:20]]).contiguous()
    lab, mind = run_assign(kl, Xh.cuda(), Ch.cuda())
    lo, mo, _ = oracle.assign(Xh.numpy(), Ch.numpy())
    np.testing.assert_array_equal(lab, lo)
    np.testing.assert_array_equal(mind.astype(np.float64), mo)


def test_small_workload_with_gpu_seeds(kl):
    w = kmpp_synth.small()
    X = w.X.cuda()
    idx, C, D, ws = kl.kmpp_seed(X, w.K, 0)
    lab, mind = run_assign(kl, X, C)
    check_assign(w.X.numpy(), C.cpu().numpy(), lab, mind)
    # the final D of the seed loop is the assignment's nearest distance
    np.testing.assert_allclose(mind, D.cpu().numpy(), rtol=2e-5, atol=0)


def test_plain_workload_full_size(kl):
    w = kmpp_synth.plain(device="cuda")
    idx, C, D, ws = kl.kmpp_seed(w.X, w.K, 0)
    print("plain workload assign", flush=True)
    lab, mind = run_assign(kl, w.X, C)
    nd = check_assign(w.X.cpu().numpy(), C.cpu().numpy(), lab, mind)
    print("labels differing at accepted near-ties:", nd, flush=True)


@pytest.mark.parametrize("d", [8, 32, 64, 100, 128, 256])
def test_bf16_rows(kl, d):
    N, K = 4_001, 300
    Xh = kmpp_synth.gaussian(N, d, seed=50 + d)
    Ch = Xh[:K].clone()
    q, _ = kl.kmpp_quantize(Xh.cuda(), kl.KMPP_BF16)
    lab, mind = run_assign(kl, q, Ch.cuda(), dtype=kl.KMPP_BF16)
    Xd = oracle.bf16_decode(oracle.bf16_encode(Xh.numpy()))
    check_assign(Xd, Ch.numpy(), lab, mind)


@pytest.mark.parametrize("d", [16, 33, 64, 128])
def test_fp8_rows(kl, d):
    N, K = 4_001, 300
    Xh = kmpp_synth.gaussian(N, d, seed=70 + d, scale=7.0)
    Ch = Xh[:K].clone()
    q, e = kl.kmpp_quantize(Xh.cuda(), kl.KMPP_FP8_E4M3)
    lab, mind = run_assign(kl, q, Ch.cuda(), X_exp=e, dtype=kl.KMPP_FP8_E4M3)
    qo, eo = oracle.fp8_quantize_rows(Xh.numpy())
    Xd = oracle.fp8_dequantize_rows(qo, eo)
    check_assign(Xd, Ch.numpy(), lab, mind)


def test_unitsphere_bf16_sample(kl):
    # the 128-d unit-sphere shape at reduced N, BF16 rows on the matrix cores
    w = kmpp_synth.unitsphere(device="cuda", N=200_000, K=1024)
    q, _ = kl.kmpp_quantize(w.X, kl.KMPP_BF16)
    C = w.X[:1024].clone()
    lab, mind = run_assign(kl, q, C, dtype=kl.KMPP_BF16)
    Xd = oracle.bf16_decode(oracle.bf16_encode(w.X.cpu().numpy()))
    check_assign(Xd, C.cpu().numpy(), lab, mind)


@pytest.mark.parametrize("K", [20, 300])
@pytest.mark.parametrize("d", [8, 32, 300])
def test_nan_row_gets_label_minus_one(kl, d, K):
    # a row with a NaN has no comparable distance: label -1, distance NaN;
    # every other row is unaffected (K = 300 spreads a short recheck queue's
    # centre tiles over several workgroups for d <= 128)
    N = 3000
    Xh = kmpp_synth.gaussian(N, d, seed=77 + d)
    Ch = Xh[:K].clone()
    Xh[123, d // 2] = float("nan")
    lab, mind = run_assign(kl, Xh.cuda(), Ch.cuda())
    assert lab[123] == -1 and np.isnan(mind[123])
    keep = np.arange(N) != 123
    check_assign(Xh.numpy()[keep], Ch.numpy(), lab[keep], mind[keep])


@pytest.mark.parametrize("dtype", [0, 1])
def test_large_norm_centres_near_rows(kl, dtype):
    # every centre and row sits near one far point (coordinates ~1000), so
    # ||c||^2 ~ 6.4e7 dwarfs every distance (~1e2): the score form's error
    # bound must carry the rounding of ||c||^2 and route these rows to the
    # direct-form recheck; labels must still match the FP64 oracle
    N, d, K = 20_011, 64, 64
    base = 1000.0
    g = torch.Generator().manual_seed(17)
    Ch = (base + torch.randn((K, d), generator=g)).float()
    Xh = (base + torch.randn((N, d), generator=g)).float()
    print("assign large-norm centres", dtype, flush=True)
    if dtype == 0:
        lab, mind = run_assign(kl, Xh.cuda(), Ch.cuda())
        Xd = Xh.numpy()
    else:
        q, _ = kl.kmpp_quantize(Xh.cuda(), kl.KMPP_BF16)
        lab, mind = run_assign(kl, q, Ch.cuda(), dtype=kl.KMPP_BF16)
        Xd = oracle.bf16_decode(oracle.bf16_encode(Xh.numpy()))
    check_assign(Xd, Ch.numpy(), lab, mind)


@pytest.mark.parametrize("N", [30_011, 70_001])
def test_recheck_queue_short_and_long(kl, N):
    # every row near one far point: the matrix-core bound decides none of
    # them, so all go to the direct-form recheck (queues of 30,011 and
    # 70,001 rows, more than one pass of the recheck grid)
    d, K = 64, 300
    g = torch.Generator().manual_seed(N)
    Ch = (500.0 + torch.randn((K, d), generator=g)).float()
    Xh = (500.0 + torch.randn((N, d), generator=g)).float()
    print("assign recheck queue", N, flush=True)
    lab, mind = run_assign(kl, Xh.cuda(), Ch.cuda())
    check_assign(Xh.numpy(), Ch.numpy(), lab, mind)


@pytest.mark.parametrize("dtype", [1, 2])
@pytest.mark.parametrize("d", [64, 128])
def test_first_stage_bound_covers_high_part_rounding(kl, dtype, d):
    # Rounding a centre value to its BF16 high part (8 significant bits,
    # nearest even) can move it by 2^-8 of itself, so the first stage's
    # products can misjudge the gap between two centres by 2^-7 |x| max|c|.
    # Rows of ones; centre 0 has every value at 1 + 3 * 2^-8 (its high part
    # rounds up, to 1 + 2^-6), centre 5 at 1 + 2^-8 (rounds down, to 1), so
    # the high parts rank centre 0 first by about d / 128 in t while centre 5
    # is nine times nearer; a bound of 2^-8 |x| max|c| would decide the rows
    # for centre 0.  The other centres have centre 0's norm (the bound grows
    # with max|c|) and random signs, so they sit far from the rows of ones;
    # the other rows are Gaussian.
    K, N = 20, 3_000
    u = 2.0 ** -8
    g = torch.Generator().manual_seed(d + dtype)
    C = (1 + 3 * u) * torch.sign(torch.randn((K, d), generator=g) + 0.5)
    C[0] = 1 + 3 * u
    C[5] = 1 + u
    Xh = torch.randn((N, d), generator=g) * 3.0
    Xh[:1_000] = 1.0
    X, E = kl.kmpp_quantize(Xh.cuda(), dtype)
    print("assign first-stage bound", dtype, d, flush=True)
    lab, mind = run_assign(kl, X, C.float().cuda(), X_exp=E, dtype=dtype)
    assert np.all(lab[:1_000] == 5), np.unique(lab[:1_000])
    if dtype == 1:
        Xd = oracle.bf16_decode(oracle.bf16_encode(Xh.numpy()))
    else:
        Xd = oracle.fp8_dequantize_rows(*oracle.fp8_quantize_rows(Xh.numpy()))
    check_assign(Xd, C.float().numpy(), lab, mind)


@pytest.mark.parametrize("K", [66, 320])
@pytest.mark.parametrize("d", [16, 64])
def test_short_recheck_queue_ties_and_nan(kl, d, K):
    # every row goes to the recheck (all near one far point), and the queue
    # is short enough for its centre tiles to be split over workgroups: the
    # second half of the centres repeats the first, so each row's best
    # distance is reached in two different tile ranges and the smaller index
    # must win; a NaN row still gets label -1 (K = 66: three centre tiles,
    # the last one partial, in two ranges)
    N = 5_003
    g = torch.Generator().manual_seed(d)
    Ch = (500.0 + torch.randn((K // 2, d), generator=g)).float()
    Ch = torch.cat([Ch, Ch]).contiguous()
    Xh = (500.0 + torch.randn((N, d), generator=g)).float()
    Xh[4_321, 3] = float("nan")
    print("assign short recheck queue ties", d, K, flush=True)
    for out_mind in (None, False):
        lab, mind, _ = kl.kmpp_assign(Xh.cuda(), Ch.cuda(), out_mind=out_mind)
        torch.cuda.synchronize()
        lab = lab.cpu().numpy()
        assert lab[4_321] == -1
        keep = np.arange(N) != 4_321
        assert np.all((lab[keep] >= 0) & (lab[keep] < K // 2))
        if mind is not None:
            mind = mind.cpu().numpy()
            assert np.isnan(mind[4_321])
            check_assign(Xh.numpy()[keep], Ch.numpy(), lab[keep], mind[keep])


@pytest.mark.parametrize("dtype", [0, 1, 2])
@pytest.mark.parametrize("d", [16, 64, 128])
def test_labels_without_distances(kl, dtype, d):
    # no distance output (a NULL out_mind): the same labels as with it, and
    # the oracle's on the stored rows
    N, K = 20_011, 300
    Xh = kmpp_synth.gaussian(N, d, seed=d + 7, scale=3.0)
    Ch = Xh[torch.randperm(N, generator=torch.Generator().manual_seed(d))[:K]].contiguous()
    X, E = (Xh.cuda(), None) if dtype == 0 else kl.kmpp_quantize(Xh.cuda(), dtype)
    print("assign labels only", dtype, d, flush=True)
    lab1, mind1, _ = kl.kmpp_assign(X, Ch.cuda(), X_exp=E, dtype=dtype)
    lab0, mind0, _ = kl.kmpp_assign(X, Ch.cuda(), X_exp=E, dtype=dtype, out_mind=False)
    torch.cuda.synchronize()
    assert mind0 is None
    assert torch.equal(lab0, lab1)
    if dtype == 0:
        Xd = Xh.numpy()
    elif dtype == 1:
        Xd = oracle.bf16_decode(oracle.bf16_encode(Xh.numpy()))
    else:
        Xd = oracle.fp8_dequantize_rows(*oracle.fp8_quantize_rows(Xh.numpy()))
    check_assign(Xd, Ch.numpy(), lab0.cpu().numpy(), mind1.cpu().numpy())
