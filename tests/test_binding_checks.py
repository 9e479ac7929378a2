"""The Python binding checks every tensor's dtype, shape and size before it
passes a pointer to the C ABI (which cannot see them): each bad argument
raises ValueError on the CPU, before any GPU call."""
import pytest
import torch


@pytest.fixture(scope="module")
def kl():
    import paper_1908_02136_amd as k
    import os
    if not os.path.exists(k.LIB_PATH):
        pytest.skip("libkmpp.so not built")
    return k


def f32(*shape):
    return torch.zeros(shape, dtype=torch.float32)


def test_seed_rejections(kl):
    X = f32(100, 8)
    with pytest.raises(ValueError, match="2-D"):
        kl.kmpp_seed(f32(100), 4)
    with pytest.raises(ValueError, match="float32"):
        kl.kmpp_seed(X.to(torch.bfloat16), 4)                      # bf16 rows with the FP32 default
    with pytest.raises(ValueError, match="dtype must be"):
        kl.kmpp_seed(X, 4, dtype=7)
    with pytest.raises(ValueError, match="Xq is required"):
        kl.kmpp_seed(X, 4, dtype=kl.KMPP_BF16)
    with pytest.raises(ValueError, match="2-byte"):
        kl.kmpp_seed(X, 4, Xq=torch.zeros((100, 8), dtype=torch.uint8), dtype=kl.KMPP_BF16)
    with pytest.raises(ValueError, match="shape"):
        kl.kmpp_seed(X, 4, Xq=torch.zeros((100, 4), dtype=torch.bfloat16), dtype=kl.KMPP_BF16)
    with pytest.raises(ValueError, match="Xq_exp"):
        kl.kmpp_seed(X, 4, Xq=torch.zeros((100, 8), dtype=torch.uint8), dtype=kl.KMPP_FP8_E4M3)
    with pytest.raises(ValueError, match="Xq_exp"):
        kl.kmpp_seed(X, 4, Xq=torch.zeros((100, 8), dtype=torch.uint8),
                     Xq_exp=torch.zeros(99, dtype=torch.int8), dtype=kl.KMPP_FP8_E4M3)
    with pytest.raises(ValueError, match="out_centers"):
        kl.kmpp_seed(X, 4, out_centers=f32(3, 8))
    with pytest.raises(ValueError, match="out_D"):
        kl.kmpp_seed(X, 4, out_D=f32(99))
    with pytest.raises(ValueError, match="out_idx"):
        kl.kmpp_seed(X, 4, out_idx=torch.zeros(4, dtype=torch.int32))
    with pytest.raises(ValueError, match="out_recheck"):
        kl.kmpp_seed(X, 4, out_recheck=f32(7))
    with pytest.raises(ValueError, match="out_sumD"):
        kl.kmpp_seed(X, 4, out_sumD=f32(4))
    # every check passed: only the device is wrong
    with pytest.raises(ValueError, match="CUDA"):
        kl.kmpp_seed(X, 4)


def test_noalloc_rejections(kl):
    X = f32(100, 8)
    with pytest.raises(ValueError, match="out_centers is required"):
        kl.kmpp_seed_noalloc(X, 4, out_centers=None)
    with pytest.raises(ValueError, match="out_status"):
        kl.kmpp_seed_noalloc(X, 4, out_centers=f32(4, 8), out_status=torch.zeros(2, dtype=torch.int32))
    with pytest.raises(ValueError, match="out_D"):
        kl.kmpp_seed_noalloc(X, 4, out_centers=f32(4, 8), out_D=f32(100, 2))


def test_assign_rejections(kl):
    X = f32(100, 8)
    C = f32(5, 8)
    with pytest.raises(ValueError, match=r"\[K, 8\]"):
        kl.kmpp_assign(X, f32(5, 7))                               # fewer centre columns than d
    with pytest.raises(ValueError, match="float32"):
        kl.kmpp_assign(X, C.double())
    with pytest.raises(ValueError, match="4-byte"):
        kl.kmpp_assign(X.to(torch.bfloat16), C)                    # BF16 rows with the FP32 default
    with pytest.raises(ValueError, match="2-byte"):
        kl.kmpp_assign(X, C, dtype=kl.KMPP_BF16)                   # FP32 rows declared BF16
    with pytest.raises(ValueError, match="X_exp"):
        kl.kmpp_assign(torch.zeros((100, 8), dtype=torch.uint8), C, dtype=kl.KMPP_FP8_E4M3)
    with pytest.raises(ValueError, match="out_labels"):
        kl.kmpp_assign(X, C, out_labels=torch.zeros(100, dtype=torch.int64))
    with pytest.raises(ValueError, match="out_mind"):
        kl.kmpp_assign(X, C, out_mind=f32(50))
    with pytest.raises(ValueError, match="CUDA"):
        kl.kmpp_assign(X, C)


def test_lloyd_quantize_kmpar_probe_rejections(kl):
    X = f32(100, 8)
    C = f32(5, 8)
    with pytest.raises(ValueError, match="out_cost"):
        kl.kmpp_lloyd(X, C, 3, out_cost=torch.zeros(2, dtype=torch.float64))
    with pytest.raises(ValueError, match="out_counts"):
        kl.kmpp_lloyd(X, C, 3, out_counts=torch.zeros(4, dtype=torch.int32))
    with pytest.raises(ValueError, match=r"\[K, 8\]"):
        kl.kmpp_lloyd(X, f32(5, 9), 1)
    with pytest.raises(ValueError, match="KMPP_BF16 or KMPP_FP8"):
        kl.kmpp_quantize(X, kl.KMPP_F32)
    with pytest.raises(ValueError, match="float32"):
        kl.kmpp_quantize(X.double(), kl.KMPP_BF16)
    with pytest.raises(ValueError, match="float32"):
        kl.kmpp_seed_parallel(X.half(), 4)
    with pytest.raises(ValueError, match="out_centers"):
        kl.kmpp_seed_parallel(X, 4, out_centers=f32(4, 7))
    with pytest.raises(ValueError, match="out"):
        kl.kmpp_read_probe(X, blocks=8, out=f32(4))


def test_batched_rejections(kl):
    Xs = [f32(100, 8), f32(50, 16)]
    with pytest.raises(ValueError, match="one K"):
        kl.kmpp_seed_batched(Xs, [4])
    with pytest.raises(ValueError, match="float32"):
        kl.kmpp_seed_batched([Xs[0].double(), Xs[1]], [4, 4])
    bad = [(f32(4, 8), f32(100), torch.zeros(4, dtype=torch.int64)),
           (f32(4, 15), f32(50), torch.zeros(4, dtype=torch.int64))]
    with pytest.raises(ValueError, match=r"outs\[1\]\[0\]"):
        kl.kmpp_seed_batched(Xs, [4, 4], outs=bad)
    with pytest.raises(ValueError, match="at least one"):
        kl.kmpp_seed_batched([], [])


def test_noalloc_c_rejections(kl):
    # argument checks of the allocation-free entry point, before any HIP call
    import ctypes
    L = kl.lib_noalloc()
    fake = ctypes.c_void_p(1 << 20)
    big = kl.NOALLOC_MAX_N + 1
    assert L.kmpp_seed_noalloc(fake, big, 2, 1, 0, fake, None, None, None, None, 0, None, None, None) == \
        kl.E_TOO_LARGE
    assert L.kmpp_seed_noalloc(fake, 10, 2, 11, 0, fake, None, None, None, None, 0, None, None, None) == -1
    assert L.kmpp_seed_noalloc(None, 10, 2, 1, 0, fake, None, None, None, None, 0, None, None, None) == -1
    assert L.kmpp_seed_noalloc(fake, 10, 2, 1, 0, fake, None, None, None, None, 1, None, None, None) == -1
    assert kl.strerror(kl.E_TOO_LARGE) != "unknown status"
