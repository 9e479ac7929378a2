"""A seeded sweep of random shapes through every entry point, each checked
against the oracle with the same rules as the dedicated tests: seeding
(FP32 / BF16 / FP8), assignment, Lloyd and k-means||.  Sizes stay small so
the oracle replays every case in full."""
import numpy as np
import pytest
import torch

import kmpp_synth
import oracle
from gpu_util import check_seed_run

pytestmark = pytest.mark.gpu

rng = np.random.default_rng(2026)
CASES = [(int(rng.integers(1, 30_000)), int(rng.choice([1, 2, 3, 5, 8, 13, 16, 31, 32, 48, 64, 96, 128, 200])),
          int(rng.integers(1, 40)), int(rng.integers(0, 3)), int(rng.integers(0, 1 << 30))) for _ in range(24)]


@pytest.fixture(scope="module")
def kl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_02136_amd as k
    k.lib()
    return k


@pytest.mark.parametrize("N,d,K,fmt,seed", CASES)
def test_sweep(kl, N, d, K, fmt, seed):
    K = min(K, N)
    print("sweep", N, d, K, fmt, seed, flush=True)
    Xh = kmpp_synth.gaussian(N, d, seed=seed % 1000, scale=float(1 + seed % 7))
    X = Xh.cuda()
    Xn = Xh.numpy()
    dt = [kl.KMPP_F32, kl.KMPP_BF16, kl.KMPP_FP8_E4M3][fmt]
    Xq = E = None
    Xd = Xn
    if dt == kl.KMPP_BF16:
        Xq, E = kl.kmpp_quantize(X, dt)
        Xd = oracle.bf16_decode(oracle.bf16_encode(Xn))
    elif dt == kl.KMPP_FP8_E4M3:
        Xq, E = kl.kmpp_quantize(X, dt)
        Xd = oracle.fp8_dequantize_rows(*oracle.fp8_quantize_rows_fast(Xn))
    # seeding
    idx, C, D, ws = kl.kmpp_seed(X, K, seed, Xq=Xq, Xq_exp=E, dtype=dt)
    st = kl.kmpp_status(ws)
    torch.cuda.synchronize()
    assert st >= 0
    check_seed_run(Xn, K, seed, idx.cpu().numpy(), C.cpu().numpy(), D.cpu().numpy(), Xd=Xd, zero_seed_rows=dt != 0)
    # assignment of the dequantised rows to the seeds
    Xa = X if dt == 0 else Xq
    lab, mind, _ = kl.kmpp_assign(Xa, C, X_exp=E, dtype=dt)
    torch.cuda.synchronize()
    Ch = C.cpu().numpy()
    lo, mo, _ = oracle.assign(Xd, Ch)
    lab_h = lab.cpu().numpy()
    bad = np.nonzero(lab_h != lo)[0]
    if bad.size:
        dg = oracle.pair_dist(Xd, bad, Ch, lab_h[bad])
        assert np.all(dg - mo[bad] <= 1e-5 * mo[bad])
    dsel = oracle.pair_dist(Xd, np.arange(N), Ch, lab_h)
    assert np.all(np.abs(mind.cpu().numpy() - dsel) <= 2e-5 * dsel + 1e-30)
    # one Lloyd iteration from the seeds
    C2, lab2, cost, ch, cnt, _ = kl.kmpp_lloyd(Xa, C.clone(), 1, X_exp=E, dtype=dt)
    torch.cuda.synchronize()
    lab2h = lab2.cpu().numpy()
    C_or, n_or = oracle.lloyd_update(Xd, lab2h, Ch)
    np.testing.assert_array_equal(cnt.cpu().numpy(), n_or)
    err = np.abs(C2.cpu().numpy().astype(np.float64) - C_or)
    tol = np.spacing(np.abs(C_or)).astype(np.float64) + float(np.abs(Xd).max()) * 2.0 ** (np.ceil(np.log2(max(N, 2))) - 61)
    assert np.all(err <= tol)
    # k-means|| on FP32 rows
    if fmt == 0:
        rounds, ell = 3, 2.0 * K
        pi, pc, cand, rend, wts, plab, pws = kl.kmpp_seed_parallel(X, K, seed, rounds=rounds, ell=ell)
        pst = kl.kmpp_status(pws)
        torch.cuda.synchronize()
        assert pst >= 0
        rend = rend.cpu().numpy().astype(np.int64)
        m = int(rend[-1])
        cand_h = cand.cpu().numpy()[:m]
        r = oracle.kmpar(Xn, K, seed=seed, rounds=rounds, ell=ell, keep_D=True, replay_cand=cand_h,
                         replay_end=rend, replay_w=wts.cpu().numpy()[:m], replay_idx=pi.cpu().numpy())
        assert int(r.cand[0]) == int(cand_h[0])
        for q in range(rounds):
            mine = set(cand_h[rend[q]:rend[q + 1]].tolist())
            own = set(r.cand[r.round_end[q]:r.round_end[q + 1]].tolist())
            for i in mine ^ own:
                p = min(1.0, ell * r.Dr[q][i] / r.phi[q])
                u = oracle.uniform4(seed, int(i), 0, q + 1, 1)
                assert abs(u - p) <= 1e-5 * p + 1e-12
        pih = pi.cpu().numpy()
        for k in range(K):
            assert oracle.seed_index_ok(int(pih[k]), r.rec[k], int(r.idx[k])), k
