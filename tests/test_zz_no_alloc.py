"""kmpp_seed_noalloc (the seed loop with the library's fixed device array
instead of a caller workspace) against kmpp_seed, through the C ABI: two
calls in a row, the second on a smaller input, each bit-identical to the
workspace entry point's seeds, centres and D (the same kernels and launch
shapes) and within the parity rules of the FP64 oracle; the status comes
back through out_status; inputs beyond the array are rejected on the host."""
import numpy as np
import pytest
import torch

import kmpp_synth
from gpu_util import check_seed_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_02136_amd as k
    k.lib()
    return k


def _noalloc(kl, X, K, seed, **kw):
    N, d = X.shape
    C = torch.full((K, d), float("nan"), device="cuda")
    D = torch.full((N,), float("nan"), device="cuda")
    idx = torch.full((K,), -1, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    kl.kmpp_seed_noalloc(X, K, seed, out_centers=C, out_D=D, out_idx=idx, out_status=st, **kw)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), C.cpu().numpy(), D.cpu().numpy(), int(st.item())


def _with_ws(kl, X, K, seed, **kw):
    idx, C, D, ws = kl.kmpp_seed(X, K, seed, **kw)
    st = kl.kmpp_status(ws)
    return idx.cpu().numpy(), C.cpu().numpy(), D.cpu().numpy(), st


def _same(a, b):
    ia, Ca, Da, sa = a
    ib, Cb, Db, sb = b
    assert sa == sb
    assert np.array_equal(ia, ib)
    assert np.array_equal(Ca.view(np.uint32), Cb.view(np.uint32))
    assert np.array_equal(Da.view(np.uint32), Db.view(np.uint32))


def test_two_calls_second_smaller(kl):
    # the 1,000,000 x 32, K = 256 workload, then the 10,000 x 2, K = 16 one
    big = kmpp_synth.plain(device="cuda")
    print("noalloc: plain N=1000000 d=32 K=256", flush=True)
    a = _noalloc(kl, big.X, big.K, 0)
    assert a[3] == 0
    _same(a, _with_ws(kl, big.X, big.K, 0))
    # (10,000 x 2 fits one workgroup's LDS: the automatic placement runs
    # the whole loop in one workgroup, on the array's status word too)
    small = kmpp_synth.small()
    print("noalloc: small N=10000 d=2 K=16 (after the large call)", flush=True)
    b = _noalloc(kl, small.X.cuda(), small.K, 3)
    assert b[3] == 0
    _same(b, _with_ws(kl, small.X.cuda(), small.K, 3))
    check_seed_run(small.X.numpy(), small.K, 3, b[0], b[1], b[2])
    # the first call against the oracle too (every draw replayed, every D)
    check_seed_run(big.X.cpu().numpy(), big.K, 0, a[0], a[1], a[2])


def test_both_draw_placements_and_bf16(kl):
    Xh = kmpp_synth.gaussian(60_013, 64, seed=11, scale=3.0)
    X = Xh.cuda()
    for draw in (kl.KMPP_DRAW_PASS, kl.KMPP_DRAW_KERNEL, kl.KMPP_DRAW_LEAD):
        print("noalloc: gaussian 60013 x 64, draw", draw, flush=True)
        a = _noalloc(kl, X, 40, 5, draw=draw)
        _same(a, _with_ws(kl, X, 40, 5, draw=draw))
        check_seed_run(Xh.numpy(), 40, 5, a[0], a[1], a[2])
    q, _ = kl.kmpp_quantize(X, kl.KMPP_BF16)
    print("noalloc: the same rows in BF16", flush=True)
    a = _noalloc(kl, X, 40, 5, Xq=q, dtype=kl.KMPP_BF16)
    _same(a, _with_ws(kl, X, 40, 5, Xq=q, dtype=kl.KMPP_BF16))


def test_status_and_limits(kl):
    # fewer distinct rows than seeds: the warning arrives through out_status
    X = torch.ones((5_000, 4), device="cuda")
    a = _noalloc(kl, X, 8, 1)
    assert a[3] == kl.W_DEGENERATE
    assert _with_ws(kl, X, 8, 1)[3] == kl.W_DEGENERATE
    # the largest accepted input, then one row more (rejected on the host)
    N = kl.NOALLOC_MAX_N
    Xb = kmpp_synth.gaussian(N + 1, 2, device="cuda", seed=3)
    print("noalloc: N at the limit", N, flush=True)
    a = _noalloc(kl, Xb[:N], 64, 2)
    assert a[3] == 0
    _same(a, _with_ws(kl, Xb[:N].contiguous(), 64, 2))
    C = torch.empty((4, 2), device="cuda")
    with pytest.raises(kl.KmppError) as e:
        kl.kmpp_seed_noalloc(Xb, 4, 0, out_centers=C)
    assert e.value.code == kl.E_TOO_LARGE
