"""GPU parity of the precision forms: the quantisers against the oracle's
format definitions (bit-exact), and the seed loop on BF16 / per-row FP8
rows against the oracle run on the dequantised rows with FP32 centres."""
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


def _fp8_host(kl, X):
    q, e = kl.kmpp_quantize(X, kl.KMPP_FP8_E4M3)
    torch.cuda.synchronize()
    return q.view(torch.uint8).cpu().numpy(), e.cpu().numpy()


@pytest.mark.parametrize("d", [3, 16, 64, 128])
def test_bf16_quantiser_bit_exact(kl, d):
    Xh = kmpp_synth.gaussian(20_001, d, seed=d, scale=37.0)
    Xh[0, 0] = 1.00390625          # exact tie 1 + 2^-8: rounds to even (1.0)
    Xh[1, 0] = 1.01171875          # exact tie 1 + 3*2^-8: rounds to even (1.015625)
    q, _ = kl.kmpp_quantize(Xh.cuda(), kl.KMPP_BF16)
    got = q.view(torch.uint16).cpu().numpy() if hasattr(torch, "uint16") else q.view(torch.int16).cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(got, oracle.bf16_encode(Xh.numpy()))


@pytest.mark.parametrize("d,scale", [(5, 1.0), (64, 100.0), (128, 0.01), (64, 1e-30), (4, 3.0), (8, 3.0),
                                     (12, 3.0), (256, 3.0), (260, 3.0)])
def test_fp8_quantiser_bit_exact(kl, d, scale):
    Xh = kmpp_synth.gaussian(4_001, d, seed=d, scale=scale)
    Xh[3] = 0.0                    # all-zero row: exponent 0
    Xh[4, :] = 448.0               # exponent 0 exactly at the top code
    q, e = _fp8_host(kl, Xh.cuda())
    qo, eo = oracle.fp8_quantize_rows(Xh.numpy())
    np.testing.assert_array_equal(e, eo)
    np.testing.assert_array_equal(q, qo)


@pytest.mark.parametrize("d", [8, 32, 64, 100, 128])
def test_bf16_seed_parity(kl, d):
    N, K = 60_013, 24
    Xh = kmpp_synth.gaussian(N, d, seed=200 + d)
    X = Xh.cuda()
    q, _ = kl.kmpp_quantize(X, kl.KMPP_BF16)
    rec = torch.zeros(2 * K, device="cuda")
    idx, C, D, st = run_seed(kl, X, K, seed=4, Xq=q, dtype=kl.KMPP_BF16, out_recheck=rec)
    assert st == 0
    Xd = oracle.bf16_decode(oracle.bf16_encode(Xh.numpy()))
    check_seed_run(Xh.numpy(), K, 4, idx, C, D, Xd=Xd, zero_seed_rows=True)
    r = rec.cpu().numpy().reshape(K, 2)
    assert np.all(r[1:, 1] > 0) and np.all(np.isfinite(r[1:]))


@pytest.mark.parametrize("d", [16, 33, 64, 128])
def test_fp8_seed_parity(kl, d):
    N, K = 60_013, 24
    Xh = kmpp_synth.gaussian(N, d, seed=300 + d, scale=5.0)
    X = Xh.cuda()
    q, e = kl.kmpp_quantize(X, kl.KMPP_FP8_E4M3)
    idx, C, D, st = run_seed(kl, X, K, seed=5, Xq=q, Xq_exp=e, dtype=kl.KMPP_FP8_E4M3)
    assert st == 0
    qo, eo = oracle.fp8_quantize_rows(Xh.numpy())
    Xd = oracle.fp8_dequantize_rows(qo, eo)
    check_seed_run(Xh.numpy(), K, 5, idx, C, D, Xd=Xd, zero_seed_rows=True)


@pytest.mark.parametrize("fmt,d", [("bf16", 32), ("bf16", 64), ("fp8", 64), ("fp8", 128)])
def test_precision_forms_draw_placements(kl, fmt, d):
    # the draw at the start of the next pass, the draw kernel and the lead
    # workgroup's draw at 256 threads: the same seeds, D and recheck values,
    # and against the oracle on the dequantised rows
    N, K = 60_013, 24
    Xh = kmpp_synth.gaussian(N, d, seed=400 + d, scale=5.0)
    X = Xh.cuda()
    dt = kl.KMPP_BF16 if fmt == "bf16" else kl.KMPP_FP8_E4M3
    q, e = kl.kmpp_quantize(X, dt)
    out = []
    for draw in (kl.KMPP_DRAW_PASS, kl.KMPP_DRAW_KERNEL, kl.KMPP_DRAW_LEAD):
        rec = torch.zeros(2 * K, device="cuda")
        idx, C, D, st = run_seed(kl, X, K, seed=6, Xq=q, Xq_exp=e, dtype=dt, out_recheck=rec, threads=256,
                                 draw=draw)
        assert st == 0
        out.append((idx, C, D, rec.cpu().numpy()))
    ia, Ca, Da, ra = out[0]
    for ib, Cb, Db, rb in out[1:]:
        assert np.array_equal(ia, ib)
        assert np.array_equal(Da.view(np.uint32), Db.view(np.uint32))
        assert np.array_equal(ra.view(np.uint32), rb.view(np.uint32))
    if fmt == "bf16":
        Xd = oracle.bf16_decode(oracle.bf16_encode(Xh.numpy()))
    else:
        Xd = oracle.fp8_dequantize_rows(*oracle.fp8_quantize_rows(Xh.numpy()))
    check_seed_run(Xh.numpy(), K, 6, ia, Ca, Da, Xd=Xd, zero_seed_rows=True)
