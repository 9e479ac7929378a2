"""The C ABI on the CPU: the library loads, exports every function that
include/kmpp.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def kl():
    import paper_1908_02136_amd as k
    if not os.path.exists(k.LIB_PATH):
        pytest.skip("libkmpp.so not built")
    k.lib()
    return k


def _declared():
    txt = open(os.path.join(ROOT, "include", "kmpp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(kmpp_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported(kl):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        # the allocation-free entry point is exported by its own library
        owner = kl.lib_noalloc() if n in kl.NOALLOC_SYMBOLS else kl.lib()
        assert hasattr(owner, n), n
    assert sorted(kl.SYMBOLS) == names


def test_strerror_and_version(kl):
    assert kl.kmpp_version() >= 100
    for c in [0, 1, -1, -2, -3, -4, -5, -6]:
        assert kl.strerror(c) and kl.strerror(c) != "unknown status"


def test_workspace_sizes(kl):
    L = kl.lib()
    assert L.kmpp_seed_workspace_bytes(0, 4, 1, 0) == 0
    assert L.kmpp_seed_workspace_bytes(10, 4, 11, 0) == 0
    assert L.kmpp_seed_workspace_bytes(10, 5000, 1, 0) == 0
    assert L.kmpp_seed_workspace_bytes(10, 4, 1, 7) == 0
    a = L.kmpp_seed_workspace_bytes(1_000_000, 32, 256, 0)
    assert a >= 256 + 4 * 1_000_000 + 8 * 256
    assert a % 256 == 0


def test_seed_argument_checks_need_no_gpu(kl):
    L = kl.lib()
    fake = ctypes.c_void_p(1 << 20)       # never dereferenced: validation fails first
    ws = ctypes.c_void_p(1 << 21)
    # N < K
    assert L.kmpp_seed(fake, 10, 2, 11, 0, fake, None, None, None, None, 0, None, ws, 1 << 30, None) == -1
    # d out of range
    assert L.kmpp_seed(fake, 10, 0, 1, 0, fake, None, None, None, None, 0, None, ws, 1 << 30, None) == -1
    assert L.kmpp_seed(fake, 10, 5000, 1, 0, fake, None, None, None, None, 0, None, ws, 1 << 30, None) == -1
    # misaligned X
    assert L.kmpp_seed(ctypes.c_void_p((1 << 20) + 4), 10, 2, 1, 0, fake, None, None, None, None, 0, None, ws,
                       1 << 30, None) == -1
    # precision form without quantised rows / exponents
    assert L.kmpp_seed(fake, 10, 2, 1, 0, fake, None, None, None, None, 1, None, ws, 1 << 30, None) == -1
    assert L.kmpp_seed(fake, 10, 2, 1, 0, fake, None, None, fake, None, 2, None, ws, 1 << 30, None) == -1
    # small workspace
    assert L.kmpp_seed(fake, 10, 2, 1, 0, fake, None, None, None, None, 0, None, ws, 16, None) == -2
    # null outputs
    assert L.kmpp_seed(fake, 10, 2, 1, 0, None, None, None, None, None, 0, None, ws, 1 << 30, None) == -1
    # unknown draw mode
    opts = kl.SeedOpts(0, 0, 0, 0, -1, None, None, 0, 5)
    assert L.kmpp_seed(fake, 10, 2, 1, 0, fake, None, None, None, None, 0, ctypes.byref(opts), ws, 1 << 30,
                       None) == -1


def test_other_argument_checks_need_no_gpu(kl):
    L = kl.lib()
    fake = ctypes.c_void_p(1 << 20)
    assert L.kmpp_quantize(fake, 10, 4, 0, fake, None, None) == -1          # F32 is not a storage target
    assert L.kmpp_quantize(fake, 10, 4, 2, fake, None, None) == -1          # FP8 needs exponents
    assert L.kmpp_assign(None, None, 0, fake, 10, 4, 3, fake, None, fake, 1 << 30, None) == -1
    assert L.kmpp_assign(fake, None, 2, fake, 10, 4, 3, fake, None, fake, 1 << 30, None) == -1
    assert L.kmpp_seed_batched(None, 3, 0, fake, 1 << 30, None) == -1
    assert L.kmpp_status(None, None, None) == -1
    assert L.kmpp_tune_load(b"/nonexistent/file") == -1
    # read probe: size not a multiple of 16, no workgroups, bad load kind, null output
    assert L.kmpp_read_probe(fake, 100, 4, 0, fake, None) == -1
    assert L.kmpp_read_probe(fake, 1024, 0, 0, fake, None) == -1
    assert L.kmpp_read_probe(fake, 1024, 4, 2, fake, None) == -1
    assert L.kmpp_read_probe(fake, 1024, 4, 0, None, None) == -1


def test_single_workgroup_limits_need_no_gpu(kl):
    # KMPP_DRAW_SINGLE refuses what one workgroup cannot hold (more than 36
    # interleaved values per thread, more than 16384 rows, stored rows, a
    # pass option) before any HIP call
    L = kl.lib()
    fake = ctypes.c_void_p(1 << 20)
    ws = ctypes.c_void_p(1 << 24)
    for N, d, kw, dtype in ((3_000, 13, {}, 0), (16_385, 1, {}, 0), (1_000, 8, {"threads": 256}, 0),
                            (1_000, 8, {}, 1)):
        opts = kl.SeedOpts(0, kw.get("threads", 0), 0, 0, -1, None, None, 0, kl.KMPP_DRAW_SINGLE)
        xq = fake if dtype else None
        assert L.kmpp_seed(fake, N, d, 4, 0, fake, None, None, xq, None, dtype, ctypes.byref(opts), ws, 1 << 30,
                           None) == kl.E_UNSUPPORTED, (N, d, kw, dtype)


def test_batched_dtype_checks_need_no_gpu(kl):
    # a batch streams one row format; BF16 / FP8 instances need their stored
    # rows (and FP8 its exponents); all refused before any HIP call (the
    # pointers are never dereferenced on these paths)
    fake = 1 << 20  # 16-byte aligned stand-in address
    def inst(dtype, xq=fake, xe=fake):
        return kl.Instance(fake, 1_000, 16, 4, fake, None, None, dtype, xq, xe)
    L = kl.lib()
    mixed = (kl.Instance * 2)(inst(0, None, None), inst(1))
    assert L.kmpp_batched_workspace_bytes(mixed, 2) == 0
    assert L.kmpp_seed_batched_prepare(mixed, 2, 0, fake, 1 << 30, None) == kl.E_UNSUPPORTED
    for bad in (inst(1, xq=None), inst(1, xq=fake + 8), inst(2, xe=None), inst(7)):
        one = (kl.Instance * 1)(bad)
        assert L.kmpp_seed_batched_prepare(one, 1, 0, fake, 1 << 30, None) == kl.E_INVALID
    with pytest.raises(ValueError, match="Xq"):
        kl._instances([_cpu_rows()], [4], [(None, None, None)], kl.KMPP_BF16)


def _cpu_rows():
    import torch
    return torch.zeros((10, 16))


def test_tune_file_parses(kl, tmp_path):
    p = tmp_path / "t.txt"
    p.write_text("seed 0 32 256 512\nseed 0 64 512 256\n# comment\nseed 9 1 256 1\nbogus\n"
                 # the draw column: 1 (at pass start), 2 (kernel), 3 (lead workgroup); 4 and -1 are rejected
                 "seed 0 8 256 1024 16 1 1\nseed 0 16 512 1024 8 1 2\nseed 0 32 512 1024 8 1 3\n"
                 "seed 0 4 256 1024 8 0 4\nseed 0 4 256 1024 8 0 -1\n"
                 # the lead workgroup's wait budget
                 "lead wait_ms 250\nlead budget 3\n")
    q = tmp_path / "lead_default.txt"
    q.write_text("lead wait_ms -1\n")
    try:
        assert kl.lib().kmpp_tune_load(str(p).encode()) == 6
    finally:
        kl.lib().kmpp_tune_load(kl.TUNE_PATH.encode())  # the shipped table again
        kl.lib().kmpp_tune_load(str(q).encode())        # and the default lead-wait budget
