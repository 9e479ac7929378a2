"""GPU parity of the seed loop (paper, Section II, Algorithms 1-2) against
the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import kmpp_synth
import oracle
from gpu_util import check_seed_run, run_seed

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


def test_small_workload_full_parity(kl):
    w = kmpp_synth.small()
    _say("small workload N=10000 d=2 K=16")
    X = w.X.cuda()
    for seed in range(8):
        idx, C, D, st = run_seed(kl, X, w.K, seed)
        assert st == 0
        check_seed_run(w.X.numpy(), w.K, seed, idx, C, D)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 8])
def test_integer_lattice_is_bit_exact(kl, d):
    # integer coordinates in [-100, 100]: every distance is an integer < 2^24
    # (exact in FP32) and every FP64 sum is exact, so seeds and D must match
    # the oracle exactly
    N, K = 50_000 + 17, 40
    Xh = kmpp_synth.lattice(N, d, seed=d)
    _say("lattice", N, d, K)
    idx, C, D, st = run_seed(kl, Xh.cuda(), K, seed=3)
    assert st == 0
    check_seed_run(Xh.numpy(), K, 3, idx, C, D, exact=True)


@pytest.mark.parametrize("d", [1, 3, 4, 5, 8, 16, 17, 32, 33, 64, 100, 127, 128, 256, 300, 512, 1000])
def test_shapes_ragged_tiles(kl, d):
    N = 70_001
    K = 12
    Xh = kmpp_synth.gaussian(N, d, seed=100 + d)
    _say("gaussian", N, d, K)
    idx, C, D, st = run_seed(kl, Xh.cuda(), K, seed=d)
    assert st == 0
    check_seed_run(Xh.numpy(), K, d, idx, C, D)


@pytest.mark.parametrize("threads,rpt", [(256, 0), (512, 0), (256, 64), (512, 1024), (256, 5000)])
def test_launch_shapes(kl, threads, rpt):
    N, d, K = 123_457, 32, 20
    Xh = kmpp_synth.gaussian(N, d, seed=5)
    _say("launch", threads, rpt)
    idx, C, D, st = run_seed(kl, Xh.cuda(), K, seed=1, threads=threads, rows_per_tile=rpt)
    assert st == 0
    check_seed_run(Xh.numpy(), K, 1, idx, C, D)


@pytest.mark.parametrize("threads,rpt,K", [(256, 0, 24), (256, 64, 24), (512, 0, 24), (512, 512, 300),
                                           (256, 5000, 24)])
def test_draw_at_pass_start_matches_draw_kernel(kl, threads, rpt, K):
    # the draw by every workgroup at the start of the next pass against the
    # draw kernel: the same fixed-order steps, so at 256 threads (the draw
    # kernel's size) the same seeds and D; at 512 threads both against the
    # oracle.  rpt=64 gives 1930 tiles; rpt=5000 is too large a tile for the
    # LDS share (draw kernel in both modes)
    N, d = 123_457, 32
    Xh = kmpp_synth.gaussian(N, d, seed=11)
    X = Xh.cuda()
    _say("draw at pass start vs draw kernel", N, d, K, threads, rpt)
    a = run_seed(kl, X, K, seed=4, threads=threads, rows_per_tile=rpt, draw=kl.KMPP_DRAW_PASS)
    b = run_seed(kl, X, K, seed=4, threads=threads, rows_per_tile=rpt, draw=kl.KMPP_DRAW_KERNEL)
    assert a[3] == 0 and b[3] == 0
    if threads == 256:
        assert np.array_equal(a[0], b[0])
        assert np.array_equal(a[2], b[2])
    for idx, C, D, _ in (a, b):
        check_seed_run(Xh.numpy(), K, 4, idx, C, D)


@pytest.mark.parametrize("threads,rpt,K", [(256, 0, 24), (256, 64, 40), (512, 0, 24), (512, 512, 300),
                                           (256, 5000, 24), (512, 16, 33)])
def test_lead_draw_matches_other_placements(kl, threads, rpt, K):
    # workgroup 0 of each pass drawing for all (in place, the others waiting
    # for its index): the same fixed-order steps as the draw at pass start,
    # so the same seeds and D at any size where that one runs, the draw
    # kernel's at 256 threads, and the oracle's.  rpt=16 gives 7717 tiles
    N, d = 123_457, 32
    Xh = kmpp_synth.gaussian(N, d, seed=21)
    X = Xh.cuda()
    _say("lead draw vs other placements", N, d, K, threads, rpt)
    a = run_seed(kl, X, K, seed=5, threads=threads, rows_per_tile=rpt, draw=kl.KMPP_DRAW_LEAD)
    b = run_seed(kl, X, K, seed=5, threads=threads, rows_per_tile=rpt, draw=kl.KMPP_DRAW_KERNEL)
    assert a[3] == 0 and b[3] == 0
    if threads == 256:
        assert np.array_equal(a[0], b[0])
        assert np.array_equal(a[2], b[2])
    if rpt not in (5000, 16):  # the draw at pass start runs (LDS share, tile count)
        c = run_seed(kl, X, K, seed=5, threads=threads, rows_per_tile=rpt, draw=kl.KMPP_DRAW_PASS)
        assert np.array_equal(a[0], c[0])
        assert np.array_equal(a[2], c[2])
    check_seed_run(Xh.numpy(), K, 5, a[0], a[1], a[2])


@pytest.mark.parametrize("d,rpt", [(3, 0), (9, 0), (31, 64), (100, 0), (9, 5000)])
def test_generic_width_draw_placements(kl, d, rpt):
    # FP32 widths without an exact-width pass (one value per lane, masked
    # lanes) with the draw at pass start and the lead draw: at 256 threads
    # the same seeds and D as the draw kernel, and the oracle's.  rpt=5000
    # at d=9 leaves the draw at pass start its LDS share (tile D staged)
    N, K = 40_001, 30
    Xh = kmpp_synth.gaussian(N, d, seed=31 + d, scale=2.0)
    X = Xh.cuda()
    _say("generic width draw placements", N, d, K, rpt)
    b = run_seed(kl, X, K, seed=6, threads=256, rows_per_tile=rpt, draw=kl.KMPP_DRAW_KERNEL)
    assert b[3] == 0
    for draw in (kl.KMPP_DRAW_PASS, kl.KMPP_DRAW_LEAD):
        a = run_seed(kl, X, K, seed=6, threads=256, rows_per_tile=rpt, draw=draw)
        assert a[3] == 0
        assert np.array_equal(a[0], b[0]), draw
        assert np.array_equal(a[2], b[2]), draw
    check_seed_run(Xh.numpy(), K, 6, b[0], b[1], b[2])
    # the automatic choice (tiles shrunk for this size, draw by placement)
    c = run_seed(kl, X, K, seed=6)
    assert c[3] == 0
    check_seed_run(Xh.numpy(), K, 6, c[0], c[1], c[2])


def test_lead_draw_edge_cases_and_repeats(kl):
    # a zero sum of D (uniform draws, warning), a NaN row (error), K=1, K=2,
    # K=N, and back-to-back runs on one workspace (the published index is
    # tagged by pass and reset by each run's first kernel)
    L = kl.KMPP_DRAW_LEAD
    Xh = torch.ones((1000, 8))
    idx, C, D, st = run_seed(kl, Xh.cuda(), 5, seed=2, draw=L)
    assert st == kl.W_DEGENERATE
    assert idx.tolist() == oracle.seed(Xh.numpy(), 5, seed=2).idx.tolist()
    Xn = kmpp_synth.gaussian(1000, 8, seed=3)
    Xn[17, 2] = float("nan")
    assert run_seed(kl, Xn.cuda(), 5, seed=2, draw=L)[3] == kl.E_NONFINITE
    Xg = kmpp_synth.gaussian(5000, 8, seed=13)
    for K in (1, 2):
        idx, C, D, st = run_seed(kl, Xg.cuda(), K, seed=K, draw=L)
        assert st == 0
        check_seed_run(Xg.numpy(), K, K, idx, C, D)
    Xs = kmpp_synth.gaussian(300, 8, seed=14)
    idx, C, D, st = run_seed(kl, Xs.cuda(), 300, seed=9, draw=L)
    assert st == 0
    assert sorted(idx.tolist()) == list(range(300))
    N, d = 200_003, 32
    Xr = kmpp_synth.gaussian(N, d, seed=22)
    X = Xr.cuda()
    ws = kl.workspace(kl.kmpp_seed_workspace_bytes(N, d, 64), "cuda")
    for K, seed in ((64, 1), (7, 2), (64, 1), (2, 4)):
        _say("lead draw, repeat", K, seed)
        idx, C, D, st = run_seed(kl, X, K, seed=seed, ws=ws, draw=L)
        assert st == 0
        check_seed_run(Xr.numpy(), K, seed, idx, C, D)


def test_lead_wait_expiry_reports_timeout(kl, tmp_path):
    # the host sets a zero budget for the wait on the lead workgroup's index:
    # every other workgroup gives up at once, the passes drain normally and
    # the status says KMPP_E_TIMEOUT; with the default budget restored the
    # same seeding is the oracle's again
    N, d, K = 100_003, 32, 8
    Xh = kmpp_synth.gaussian(N, d, seed=23)
    X = Xh.cuda()
    t0 = tmp_path / "lead0.txt"
    t0.write_text("lead wait_ms 0\n")
    t1 = tmp_path / "lead_default.txt"
    t1.write_text("lead wait_ms -1\n")
    try:
        assert kl.kmpp_tune_load(str(t0)) == 1
        _say("lead draw, zero wait budget", N, d, K)
        st = run_seed(kl, X, K, seed=3, draw=kl.KMPP_DRAW_LEAD)[3]
        assert st == kl.E_TIMEOUT
    finally:
        assert kl.kmpp_tune_load(str(t1)) == 1
    idx, C, D, st = run_seed(kl, X, K, seed=3, draw=kl.KMPP_DRAW_LEAD)
    assert st == 0
    check_seed_run(Xh.numpy(), K, 3, idx, C, D)


def test_draw_at_pass_start_repeated_calls_one_workspace(kl):
    # the D and tile-sum buffers alternate by pass and the last pass writes
    # the caller's D whatever the parity of K: back-to-back runs on one
    # workspace, odd and even K, each match the oracle
    N, d = 200_003, 8
    Xh = kmpp_synth.gaussian(N, d, seed=12)
    X = Xh.cuda()
    ws = kl.workspace(kl.kmpp_seed_workspace_bytes(N, d, 64), "cuda")
    for K, seed in ((64, 1), (7, 2), (64, 3), (2, 4)):
        _say("draw at pass start, repeat", K, seed)
        idx, C, D, st = run_seed(kl, X, K, seed=seed, ws=ws)
        assert st == 0
        check_seed_run(Xh.numpy(), K, seed, idx, C, D)


def test_draw_at_pass_start_edge_cases(kl):
    # d=8 has a pass with the draw at its start: a zero sum of D (uniform
    # draws, warning), a NaN row (error), K=1 (no draw), K=2, K=N
    P = kl.KMPP_DRAW_PASS
    Xh = torch.ones((1000, 8))
    idx, C, D, st = run_seed(kl, Xh.cuda(), 5, seed=2, draw=P)
    assert st == kl.W_DEGENERATE
    r = oracle.seed(Xh.numpy(), 5, seed=2)
    assert idx.tolist() == r.idx.tolist()
    Xn = kmpp_synth.gaussian(1000, 8, seed=3)
    Xn[17, 2] = float("nan")
    assert run_seed(kl, Xn.cuda(), 5, seed=2, draw=P)[3] == kl.E_NONFINITE
    Xg = kmpp_synth.gaussian(5000, 8, seed=13)
    for K in (1, 2):
        idx, C, D, st = run_seed(kl, Xg.cuda(), K, seed=K, draw=P)
        assert st == 0
        check_seed_run(Xg.numpy(), K, K, idx, C, D)
    Xs = kmpp_synth.gaussian(300, 8, seed=14)
    idx, C, D, st = run_seed(kl, Xs.cuda(), 300, seed=9, draw=P)
    assert st == 0
    assert sorted(idx.tolist()) == list(range(300))
    assert np.all(D == 0.0)


@pytest.mark.parametrize("draw", ["pass", "kernel", "lead", "single"])
def test_graph_capture_seed_and_assign(kl, draw):
    # seeding + assignment captured into a HIP graph and replayed three
    # times, outputs cleared eagerly between replays: every replay equals
    # the eager run (the draw at pass start alternates buffers by pass, fixed
    # per captured launch)
    N, d, K = (150_001, 32, 40) if draw != "single" else (12_001, 2, 40)
    Xh = kmpp_synth.gaussian(N, d, seed=15)
    X = Xh.cuda()
    dm = {"pass": kl.KMPP_DRAW_PASS, "kernel": kl.KMPP_DRAW_KERNEL, "lead": kl.KMPP_DRAW_LEAD,
          "single": kl.KMPP_DRAW_SINGLE}[draw]
    idx = torch.empty(K, dtype=torch.int64, device="cuda")
    C = torch.empty((K, d), dtype=torch.float32, device="cuda")
    D = torch.empty(N, dtype=torch.float32, device="cuda")
    lab = torch.empty(N, dtype=torch.int32, device="cuda")
    mind = torch.empty(N, dtype=torch.float32, device="cuda")
    ws = kl.workspace(kl.kmpp_seed_workspace_bytes(N, d, K), "cuda")
    wa = kl.workspace(kl.kmpp_assign_workspace_bytes(N, d, K), "cuda")
    s = torch.cuda.Stream()

    def run():
        kl.kmpp_seed(X, K, 8, out_centers=C, out_D=D, out_idx=idx, draw=dm, ws=ws)
        kl.kmpp_assign(X, C, out_labels=lab, out_mind=mind, ws=wa)

    with torch.cuda.stream(s):
        run()
    s.synchronize()
    ref = [t.clone() for t in (idx, C, D, lab, mind)]
    with torch.cuda.stream(s):
        g = kl.Graph()
        with g.capture():
            run()
    for rep in range(3):
        for t in (idx, C, D, lab, mind):
            t.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.launch()
        s.synchronize()
        assert kl.kmpp_status(ws) == 0
        for a, b in zip((idx, C, D, lab, mind), ref):
            assert torch.equal(a, b), f"replay {rep} differs"
    check_seed_run(Xh.numpy(), K, 8, idx.cpu().numpy(), C.cpu().numpy(), D.cpu().numpy())


@pytest.mark.parametrize("N,d,K", [(10_000, 2, 16), (16_384, 1, 300), (3_001, 8, 100), (700, 23, 50),
                                   (1_000, 24, 1), (5, 3, 5), (2_048, 12, 2_048),
                                   (4_096, 9, 100), (12_000, 3, 200), (1_024, 36, 64)])
def test_single_workgroup_seeding(kl, N, d, K):
    # the whole loop in one workgroup: oracle parity (replay), the per-draw
    # sums of D, the same results under the automatic choice, and seeds that
    # mostly agree with the multi-workgroup passes (draws within rounding of
    # a row boundary may differ: each is checked against the oracle)
    Xh = kmpp_synth.gaussian(N, d, seed=N + d, scale=2.0)
    X = Xh.cuda()
    sD = torch.empty(K, dtype=torch.float64, device="cuda")
    _say("single workgroup", N, d, K)
    idx, C, D, st = run_seed(kl, X, K, seed=3, draw=kl.KMPP_DRAW_SINGLE, out_sumD=sD)
    assert st == 0
    r, _ = check_seed_run(Xh.numpy(), K, 3, idx, C, D)
    sums = sD.cpu().numpy()
    assert sums[0] == 0.0
    if K > 1:
        # the FP64 sums of the GPU's FP32 D against the oracle's FP64 totals
        np.testing.assert_allclose(sums[1:], r.rec[1:K, oracle.REC_T], rtol=1e-5)
    ia, Ca, Da, sta = run_seed(kl, X, K, seed=3)
    assert sta == 0 and np.array_equal(ia, idx) and np.array_equal(Da, D)
    ik, Ck, Dk, stk = run_seed(kl, X, K, seed=3, draw=kl.KMPP_DRAW_KERNEL)
    assert stk == 0
    assert np.mean(ik == idx) >= 0.9 or K <= 5


def test_single_workgroup_edge_cases(kl):
    S = kl.KMPP_DRAW_SINGLE
    # zero sum of D: uniform draws and the warning, as in the oracle
    Xh = torch.ones((1000, 8))
    idx, C, D, st = run_seed(kl, Xh.cuda(), 5, seed=2, draw=S)
    assert st == kl.W_DEGENERATE
    assert idx.tolist() == oracle.seed(Xh.numpy(), 5, seed=2).idx.tolist()
    # a NaN row: the error status
    Xn = kmpp_synth.gaussian(1000, 8, seed=3)
    Xn[17, 2] = float("nan")
    assert run_seed(kl, Xn.cuda(), 5, seed=2, draw=S)[3] == kl.E_NONFINITE
    # inputs it does not take: ceil(N / 1024) d > 36, more than 16384 rows,
    # stored rows, a pass option
    for shape, kw in (((3_000, 13), {}), ((16_385, 1), {}), ((1_000, 8), {"threads": 256})):
        Xb = torch.zeros(shape, device="cuda")
        with pytest.raises(kl.KmppError) as e:
            kl.kmpp_seed(Xb, 4, 0, draw=S, **kw)
        assert e.value.code == kl.E_UNSUPPORTED
    Xq, _ = kl.kmpp_quantize(torch.randn((1_000, 8), device="cuda"), kl.KMPP_BF16)
    with pytest.raises(kl.KmppError) as e:
        kl.kmpp_seed(torch.randn((1_000, 8), device="cuda"), 4, 0, Xq=Xq, dtype=kl.KMPP_BF16, draw=S)
    assert e.value.code == kl.E_UNSUPPORTED
    # back-to-back runs on one workspace
    Xg = kmpp_synth.gaussian(8_000, 3, seed=5)
    ws = kl.workspace(kl.kmpp_seed_workspace_bytes(8_000, 3, 64), "cuda")
    for K, seed in ((64, 1), (7, 2), (64, 1)):
        idx, C, D, st = run_seed(kl, Xg.cuda(), K, seed=seed, ws=ws, draw=S)
        assert st == 0
        check_seed_run(Xg.numpy(), K, seed, idx, C, D)


def test_K1_and_K_equals_N(kl):
    Xh = kmpp_synth.gaussian(300, 5, seed=6)
    idx, C, D, st = run_seed(kl, Xh.cuda(), 1, seed=9)
    check_seed_run(Xh.numpy(), 1, 9, idx, C, D)
    idx, C, D, st = run_seed(kl, Xh.cuda(), 300, seed=9)
    assert st == 0
    assert sorted(idx.tolist()) == list(range(300))
    assert np.all(D == 0.0)
    check_seed_run(Xh.numpy(), 300, 9, idx, C, D)


def test_N1(kl):
    Xh = torch.tensor([[1.5, -2.0, 3.0]])
    idx, C, D, st = run_seed(kl, Xh.cuda(), 1, seed=0)
    assert idx.tolist() == [0] and D.tolist() == [0.0]


def test_degenerate_and_nonfinite_status(kl):
    Xh = torch.ones((1000, 4))
    idx, C, D, st = run_seed(kl, Xh.cuda(), 5, seed=2)
    assert st == kl.W_DEGENERATE
    r = oracle.seed(Xh.numpy(), 5, seed=2)
    assert r.status == oracle.W_DEGENERATE
    assert idx.tolist() == r.idx.tolist()
    Xn = kmpp_synth.gaussian(1000, 4, seed=3)
    Xn[17, 2] = float("nan")
    idx, C, D, st = run_seed(kl, Xn.cuda(), 5, seed=2)
    assert st == kl.E_NONFINITE


def test_determinism_and_instance_ids(kl):
    Xh = kmpp_synth.gaussian(200_000, 16, seed=8)
    X = Xh.cuda()
    a = run_seed(kl, X, 64, seed=77)
    b = run_seed(kl, X, 64, seed=77)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2].view(np.uint32), b[2].view(np.uint32))
    c = run_seed(kl, X, 64, seed=77, instance=5)
    check_seed_run(Xh.numpy(), 64, 77, c[0], c[1], c[2], inst=5)


def test_plain_workload_full_size(kl):
    """N=1,000,000, d=32, K=256 Gaussian mixture: every draw replayed."""
    w = kmpp_synth.plain(device="cuda")
    _say("plain workload full size")
    idx, C, D, st = run_seed(kl, w.X, w.K, seed=0)
    assert st == 0
    r, differ = check_seed_run(w.X.cpu().numpy(), w.K, 0, idx, C, D)
    _say("draws differing near a boundary:", differ)


def test_argument_errors(kl):
    X = torch.zeros((10, 4), device="cuda")
    with pytest.raises(kl.KmppError) as e:
        kl.kmpp_seed(X, 11)
    assert e.value.code == kl.E_INVALID
    with pytest.raises(kl.KmppError) as e:
        kl.kmpp_seed(X, 3, ws=kl.workspace(64, "cuda"))
    assert e.value.code == kl.E_WORKSPACE
    Xm = torch.zeros(41, device="cuda")[1:].view(10, 4)      # 4-byte offset: misaligned
    with pytest.raises(kl.KmppError) as e:
        kl.kmpp_seed(Xm, 3)
    assert e.value.code == kl.E_INVALID
