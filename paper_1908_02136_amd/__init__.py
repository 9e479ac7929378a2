"""Python binding of libkmpp: k-means++ seeding and nearest-seed assignment
on MI355X (gfx950).

Argument marshalling only.  Every step of the seeding loop and of the
assignment runs in the library's HIP kernels; PyTorch supplies device memory
and the current stream.  The functions carry the C entry points' names
(``include/kmpp.h``) and take CUDA tensors; outputs are allocated here with
``torch.empty`` when not passed in.  There is no CPU fallback: if the
library is not built, or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkmpp.so")
# kmpp_seed_noalloc lives in a library of its own (linked to libkmpp.so): its
# fixed device array is loaded only by the callers of that entry point
LIB_NOALLOC_PATH = os.path.join(HERE, "libkmpp_noalloc.so")
TUNE_PATH = os.path.join(HERE, "tune_table.txt")

KMPP_F32, KMPP_BF16, KMPP_FP8_E4M3 = 0, 1, 2
DTYPES = {"f32": KMPP_F32, "bf16": KMPP_BF16, "fp8": KMPP_FP8_E4M3}
KMPP_ROWS_CACHED, KMPP_ROWS_NONTEMPORAL, KMPP_ROWS_BUFFER = 0, 1, 2
KMPP_CENTRE_LDS, KMPP_CENTRE_SCALAR, KMPP_CENTRE_GLOBAL = 1, 2, 3
ROW_PATHS = {"cached": KMPP_ROWS_CACHED, "nontemporal": KMPP_ROWS_NONTEMPORAL, "buffer": KMPP_ROWS_BUFFER}
CENTRE_SOURCES = {"lds": KMPP_CENTRE_LDS, "scalar": KMPP_CENTRE_SCALAR, "global": KMPP_CENTRE_GLOBAL}
KMPP_DRAW_AUTO, KMPP_DRAW_PASS, KMPP_DRAW_KERNEL, KMPP_DRAW_LEAD, KMPP_DRAW_SINGLE = 0, 1, 2, 3, 4
OK, W_DEGENERATE = 0, 1
E_INVALID, E_WORKSPACE, E_HIP, E_NONFINITE, E_UNSUPPORTED, E_TIMEOUT, E_TOO_LARGE = -1, -2, -3, -4, -5, -6, -7
MAX_D = 4096
NOALLOC_MAX_N = 1 << 20

# Every symbol the header declares (checked by the test suite); the last
# list's are exported by libkmpp_noalloc.so, the others by libkmpp.so.
NOALLOC_SYMBOLS = ["kmpp_seed_noalloc"]
SYMBOLS = NOALLOC_SYMBOLS + [
    "kmpp_seed_workspace_bytes", "kmpp_seed", "kmpp_assign_workspace_bytes", "kmpp_assign", "kmpp_quantize",
    "kmpp_lloyd_workspace_bytes", "kmpp_lloyd", "kmpp_seed_parallel_capacity",
    "kmpp_seed_parallel_workspace_bytes", "kmpp_seed_parallel",
    "kmpp_batched_workspace_bytes", "kmpp_seed_batched_prepare", "kmpp_seed_batched_launch",
    "kmpp_seed_batched", "kmpp_status", "kmpp_status_poll", "kmpp_graph_begin", "kmpp_graph_end", "kmpp_graph_launch",
    "kmpp_graph_destroy", "kmpp_tune_load", "kmpp_read_probe", "kmpp_strerror", "kmpp_version",
]


class KmppError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})" if what else f"{strerror(code)} ({code})")


class SeedOpts(ctypes.Structure):
    _fields_ = [("instance", ctypes.c_uint32), ("threads", ctypes.c_int32), ("rows_per_tile", ctypes.c_int32),
                ("loads_per_lane", ctypes.c_int16), ("row_loads", ctypes.c_int16),
                ("out_recheck", ctypes.c_void_p), ("step_events", ctypes.c_void_p),
                ("centre_source", ctypes.c_int32), ("draw", ctypes.c_int32), ("out_sumD", ctypes.c_void_p)]


class Instance(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("N", ctypes.c_int64), ("d", ctypes.c_int32), ("K", ctypes.c_int32),
                ("out_centers", ctypes.c_void_p), ("out_D", ctypes.c_void_p), ("out_idx", ctypes.c_void_p),
                ("dtype", ctypes.c_int32), ("Xq", ctypes.c_void_p), ("Xq_exp", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libkmpp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    L.kmpp_seed_workspace_bytes.argtypes = [i64, i32, i32, i32]
    L.kmpp_seed_workspace_bytes.restype = sz
    L.kmpp_seed.argtypes = [P, i64, i32, i32, u64, P, P, P, P, P, i32, ctypes.POINTER(SeedOpts), P, sz, P]
    L.kmpp_seed.restype = ctypes.c_int
    L.kmpp_assign_workspace_bytes.argtypes = [i64, i32, i32, i32]
    L.kmpp_assign_workspace_bytes.restype = sz
    L.kmpp_assign.argtypes = [P, P, i32, P, i64, i32, i32, P, P, P, sz, P]
    L.kmpp_assign.restype = ctypes.c_int
    L.kmpp_lloyd_workspace_bytes.argtypes = [i64, i32, i32, i32]
    L.kmpp_lloyd_workspace_bytes.restype = sz
    L.kmpp_lloyd.argtypes = [P, P, i32, i64, i32, i32, P, i32, P, P, P, P, P, sz, P]
    L.kmpp_lloyd.restype = ctypes.c_int
    L.kmpp_seed_parallel_capacity.argtypes = [i64, i32, ctypes.c_double]
    L.kmpp_seed_parallel_capacity.restype = i32
    L.kmpp_seed_parallel_workspace_bytes.argtypes = [i64, i32, i32, i32, ctypes.c_double]
    L.kmpp_seed_parallel_workspace_bytes.restype = sz
    L.kmpp_seed_parallel.argtypes = [P, i64, i32, i32, u64, i32, ctypes.c_double, ctypes.c_uint32, P, P, P, P, P,
                                     P, P, sz, P]
    L.kmpp_seed_parallel.restype = ctypes.c_int
    L.kmpp_quantize.argtypes = [P, i64, i32, i32, P, P, P]
    L.kmpp_quantize.restype = ctypes.c_int
    L.kmpp_batched_workspace_bytes.argtypes = [ctypes.POINTER(Instance), i32]
    L.kmpp_batched_workspace_bytes.restype = sz
    L.kmpp_seed_batched_prepare.argtypes = [ctypes.POINTER(Instance), i32, u64, P, sz, P]
    L.kmpp_seed_batched_prepare.restype = ctypes.c_int
    L.kmpp_seed_batched_launch.argtypes = [P, P]
    L.kmpp_seed_batched_launch.restype = ctypes.c_int
    L.kmpp_seed_batched.argtypes = [ctypes.POINTER(Instance), i32, u64, P, sz, P]
    L.kmpp_seed_batched.restype = ctypes.c_int
    L.kmpp_status.argtypes = [P, P, ctypes.POINTER(i32)]
    L.kmpp_status.restype = ctypes.c_int
    L.kmpp_status_poll.argtypes = [P, ctypes.POINTER(i32)]
    L.kmpp_status_poll.restype = ctypes.c_int
    L.kmpp_graph_begin.argtypes = [P]
    L.kmpp_graph_begin.restype = ctypes.c_int
    L.kmpp_graph_end.argtypes = [P, ctypes.POINTER(P)]
    L.kmpp_graph_end.restype = ctypes.c_int
    L.kmpp_graph_launch.argtypes = [P, P]
    L.kmpp_graph_launch.restype = ctypes.c_int
    L.kmpp_graph_destroy.argtypes = [P]
    L.kmpp_graph_destroy.restype = ctypes.c_int
    L.kmpp_tune_load.argtypes = [ctypes.c_char_p]
    L.kmpp_tune_load.restype = ctypes.c_int
    L.kmpp_strerror.argtypes = [ctypes.c_int]
    L.kmpp_strerror.restype = ctypes.c_char_p
    L.kmpp_version.argtypes = []
    L.kmpp_version.restype = ctypes.c_int
    L.kmpp_read_probe.argtypes = [P, sz, i32, i32, P, P]
    L.kmpp_read_probe.restype = ctypes.c_int
    if os.path.exists(TUNE_PATH):
        L.kmpp_tune_load(TUNE_PATH.encode())
    _lib = L
    return L


_lib_noalloc = None


def lib_noalloc() -> ctypes.CDLL:
    """Load libkmpp_noalloc.so (after libkmpp.so, which it links to)."""
    global _lib_noalloc
    if _lib_noalloc is not None:
        return _lib_noalloc
    lib()
    if not os.path.exists(LIB_NOALLOC_PATH):
        raise RuntimeError(f"{LIB_NOALLOC_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_NOALLOC_PATH)
    P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    L.kmpp_seed_noalloc.argtypes = [P, i64, i32, i32, u64, P, P, P, P, P, i32, ctypes.POINTER(SeedOpts), P, P]
    L.kmpp_seed_noalloc.restype = ctypes.c_int
    _lib_noalloc = L
    return L


def strerror(code: int) -> str:
    return lib().kmpp_strerror(int(code)).decode()


def _check(code: int, what: str) -> int:
    if code < 0:
        raise KmppError(code, what)
    return code


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _require_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("libkmpp takes contiguous CUDA (HIP) tensors")


# The C ABI takes bare pointers and cannot see a buffer's size or element
# type, so every tensor is checked here before its pointer is passed: a
# wrong dtype or a short buffer would make the kernels read or write past
# the allocation.
_ELEM_BYTES = {KMPP_F32: 4, KMPP_BF16: 2, KMPP_FP8_E4M3: 1}


def _expect(t, name, *, dtype=None, itemsize=None, shape=None, numel=None, min_numel=None, required=True):
    if t is None:
        if required:
            raise ValueError(f"{name} is required")
        return
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if itemsize is not None and t.element_size() != itemsize:
        raise ValueError(f"{name} must have {itemsize}-byte elements, got {t.element_size()} ({t.dtype})")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} elements, got {t.numel()}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name} must hold at least {min_numel} elements, got {t.numel()}")


def _rows(X, name="X"):
    if X is None or X.dim() != 2:
        raise ValueError(f"{name} must be a 2-D [N, d] tensor")
    return int(X.shape[0]), int(X.shape[1])


def _check_dtype(dtype):
    if dtype not in _ELEM_BYTES:
        raise ValueError(f"dtype must be KMPP_F32, KMPP_BF16 or KMPP_FP8_E4M3, got {dtype}")


def _check_rows(X, X_exp, dtype, name="X"):
    """Rows stored in `dtype` (FP32, BF16 or FP8 with int8 row exponents)."""
    _check_dtype(dtype)
    N, d = _rows(X, name)
    _expect(X, name, itemsize=_ELEM_BYTES[dtype])
    if dtype == KMPP_F32:
        _expect(X, name, dtype=torch.float32)
    if dtype == KMPP_FP8_E4M3:
        _expect(X_exp, f"{name}_exp", dtype=torch.int8, numel=N)
    return N, d


def _centres(C, d):
    """FP32 [K, d] centres for rows of width d; returns K."""
    if C is None or C.dim() != 2 or int(C.shape[1]) != d:
        raise ValueError(f"C must be a 2-D [K, {d}] tensor")
    _expect(C, "C", dtype=torch.float32)
    return int(C.shape[0])


def workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + max(int(nbytes), 256)]


# ---------------------------------------------------------------- seeding
def kmpp_seed_workspace_bytes(N: int, d: int, K: int, dtype: int = KMPP_F32) -> int:
    return int(lib().kmpp_seed_workspace_bytes(N, d, K, dtype))


def kmpp_seed(X: torch.Tensor, K: int, seed: int = 0, *, out_centers=None, out_D=None, out_idx=None, Xq=None,
              Xq_exp=None, dtype: int = KMPP_F32, instance: int = 0, threads: int = 0, rows_per_tile: int = 0,
              loads_per_lane: int = 0, row_loads: int = -1, centre_source: int = 0, out_recheck=None,
              out_sumD=None, step_events=None, draw: int = KMPP_DRAW_AUTO, ws=None, stream=None):
    """k-means++ seeding of the rows of X (FP32 [N, d]).  Returns
    (idx int64 [K], centers FP32 [K, d], D FP32 [N], workspace).
    ``row_loads`` (KMPP_ROWS_*) and ``centre_source`` (KMPP_CENTRE_*) pick
    the memory spaces of the passes (-1 / 0: tuned default); ``draw``
    (KMPP_DRAW_*) runs each draw at the start of the next pass (by every
    workgroup, or by its first for all) or in a kernel of its own;
    ``out_recheck`` (FP32 [2K]) and ``out_sumD`` (FP64
    [K]) receive the per-draw diagnostics described in kmpp.h."""
    N, d = _rows(X)
    _expect(X, "X", dtype=torch.float32)
    _check_dtype(dtype)
    if dtype != KMPP_F32:
        _expect(Xq, "Xq", itemsize=_ELEM_BYTES[dtype])
        _expect(Xq, "Xq", shape=(N, d))
        if dtype == KMPP_FP8_E4M3:
            _expect(Xq_exp, "Xq_exp", dtype=torch.int8, numel=N)
    dev = X.device
    out_centers = torch.empty((K, d), dtype=torch.float32, device=dev) if out_centers is None else out_centers
    out_D = torch.empty(N, dtype=torch.float32, device=dev) if out_D is None else out_D
    out_idx = torch.empty(K, dtype=torch.int64, device=dev) if out_idx is None else out_idx
    _expect(out_centers, "out_centers", dtype=torch.float32, numel=K * d)
    _expect(out_D, "out_D", dtype=torch.float32, numel=N)
    _expect(out_idx, "out_idx", dtype=torch.int64, numel=K)
    _expect(out_recheck, "out_recheck", dtype=torch.float32, min_numel=2 * K, required=False)
    _expect(out_sumD, "out_sumD", dtype=torch.float64, min_numel=K, required=False)
    _require_cuda(X, Xq, Xq_exp, out_centers, out_D, out_idx, out_recheck, out_sumD, ws)
    if ws is None:
        ws = workspace(kmpp_seed_workspace_bytes(N, d, K, dtype), dev)
    opts = SeedOpts(instance, threads, rows_per_tile, loads_per_lane, row_loads,
                    None if out_recheck is None else out_recheck.data_ptr(), step_events, centre_source, draw,
                    None if out_sumD is None else out_sumD.data_ptr())
    rc = lib().kmpp_seed(_ptr(X), N, d, K, seed, _ptr(out_centers), _ptr(out_D), _ptr(out_idx), _ptr(Xq),
                         _ptr(Xq_exp), dtype, ctypes.byref(opts), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "kmpp_seed")
    return out_idx, out_centers, out_D, ws


def kmpp_seed_noalloc(X: torch.Tensor, K: int, seed: int = 0, *, out_centers, out_D=None, out_idx=None,
                      out_status=None, Xq=None, Xq_exp=None, dtype: int = KMPP_F32, instance: int = 0,
                      draw: int = KMPP_DRAW_AUTO, stream=None):
    """kmpp_seed without a workspace (the library's fixed device array;
    N <= NOALLOC_MAX_N).  Nothing is allocated here either: the caller
    passes every output (``out_status``: int32 [1] or None)."""
    N, d = _rows(X)
    _expect(X, "X", dtype=torch.float32)
    _check_dtype(dtype)
    if dtype != KMPP_F32:
        _expect(Xq, "Xq", itemsize=_ELEM_BYTES[dtype])
        _expect(Xq, "Xq", shape=(N, d))
        if dtype == KMPP_FP8_E4M3:
            _expect(Xq_exp, "Xq_exp", dtype=torch.int8, numel=N)
    _expect(out_centers, "out_centers", dtype=torch.float32, numel=K * d)
    _expect(out_D, "out_D", dtype=torch.float32, numel=N, required=False)
    _expect(out_idx, "out_idx", dtype=torch.int64, numel=K, required=False)
    _expect(out_status, "out_status", dtype=torch.int32, numel=1, required=False)
    _require_cuda(X, Xq, Xq_exp, out_centers, out_D, out_idx, out_status)
    opts = SeedOpts(instance, 0, 0, 0, -1, None, None, 0, draw, None)
    rc = lib_noalloc().kmpp_seed_noalloc(_ptr(X), N, d, K, seed, _ptr(out_centers), _ptr(out_D), _ptr(out_idx), _ptr(Xq),
                                 _ptr(Xq_exp), dtype, ctypes.byref(opts), _ptr(out_status), _stream(stream))
    _check(rc, "kmpp_seed_noalloc")
    return out_idx, out_centers, out_D


def kmpp_status(ws: torch.Tensor, stream=None) -> int:
    out = ctypes.c_int32(0)
    _check(lib().kmpp_status(_ptr(ws), _stream(stream), ctypes.byref(out)), "kmpp_status")
    return int(out.value)


def kmpp_status_poll(ws: torch.Tensor) -> int:
    """The status word, read without synchronising a stream: call it after
    waiting for the work that wrote it (e.g. torch.cuda.synchronize())."""
    out = ctypes.c_int32(0)
    _check(lib().kmpp_status_poll(_ptr(ws), ctypes.byref(out)), "kmpp_status_poll")
    return int(out.value)


# ---------------------------------------------------------------- formats
def kmpp_quantize(X: torch.Tensor, dtype: int, stream=None):
    """Returns (Xq, Xq_exp): torch.bfloat16 [N, d] (exp None) or torch.float8_e4m3fn
    [N, d] with int8 [N] row exponents."""
    N, d = _rows(X)
    _expect(X, "X", dtype=torch.float32)
    if dtype not in (KMPP_BF16, KMPP_FP8_E4M3):
        raise ValueError("kmpp_quantize stores KMPP_BF16 or KMPP_FP8_E4M3 rows")
    _require_cuda(X)
    if dtype == KMPP_BF16:
        Xq = torch.empty((N, d), dtype=torch.bfloat16, device=X.device)
        E = None
    else:
        Xq = torch.empty((N, d), dtype=torch.float8_e4m3fn, device=X.device)
        E = torch.empty(N, dtype=torch.int8, device=X.device)
    _check(lib().kmpp_quantize(_ptr(X), N, d, dtype, _ptr(Xq), _ptr(E), _stream(stream)), "kmpp_quantize")
    return Xq, E


# ---------------------------------------------------------------- assignment
def kmpp_assign_workspace_bytes(N: int, d: int, K: int, dtype: int = KMPP_F32) -> int:
    return int(lib().kmpp_assign_workspace_bytes(N, d, K, dtype))


def kmpp_assign(X: torch.Tensor, C: torch.Tensor, *, X_exp=None, dtype: int = KMPP_F32, out_labels=None,
                out_mind=None, ws=None, stream=None):
    """Nearest seed of every row.  X is [N, d] in `dtype` (FP32, BF16 as
    uint16, FP8 as uint8 with X_exp).  Returns (labels int32 [N], mind FP32
    [N], ws); out_mind=False asks for the labels alone (mind is then None)."""
    N, d = _check_rows(X, X_exp, dtype)
    K = _centres(C, d)
    dev = X.device
    out_labels = torch.empty(N, dtype=torch.int32, device=dev) if out_labels is None else out_labels
    if out_mind is False:
        out_mind = None
    else:
        out_mind = torch.empty(N, dtype=torch.float32, device=dev) if out_mind is None else out_mind
        _expect(out_mind, "out_mind", dtype=torch.float32, numel=N)
    _expect(out_labels, "out_labels", dtype=torch.int32, numel=N)
    _require_cuda(X, C, X_exp, out_labels, out_mind, ws)
    if ws is None:
        ws = workspace(kmpp_assign_workspace_bytes(N, d, K, dtype), dev)
    rc = lib().kmpp_assign(_ptr(X), _ptr(X_exp), dtype, _ptr(C), N, d, K, _ptr(out_labels), _ptr(out_mind),
                           _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "kmpp_assign")
    return out_labels, out_mind, ws


# ---------------------------------------------------------------- k-means||
def kmpp_seed_parallel(X: torch.Tensor, K: int, seed: int = 0, *, rounds: int = 5, ell: float | None = None,
                       instance: int = 0, out_centers=None, ws=None, stream=None):
    """k-means|| seeding of the rows of X (FP32 [N, d], d <= 128).  Returns
    (idx int64 [K], centers FP32 [K, d], cand int64 [cap], round_end int32
    [rounds+1], weights int32 [cap], labels int32 [N], ws)."""
    N, d = _rows(X)
    _expect(X, "X", dtype=torch.float32)
    ell = float(2 * K) if ell is None else float(ell)
    dev = X.device
    cap = int(lib().kmpp_seed_parallel_capacity(N, rounds, ell))
    out_centers = torch.empty((K, d), dtype=torch.float32, device=dev) if out_centers is None else out_centers
    _expect(out_centers, "out_centers", dtype=torch.float32, numel=K * d)
    _require_cuda(X, out_centers, ws)
    idx = torch.empty(K, dtype=torch.int64, device=dev)
    cand = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    rend = torch.empty(rounds + 1, dtype=torch.int32, device=dev)
    w = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    lab = torch.empty(N, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(kmpp_seed_parallel_workspace_bytes(N, d, K, rounds, ell), dev)
    rc = lib().kmpp_seed_parallel(_ptr(X), N, d, K, seed, rounds, ell, instance, _ptr(out_centers), _ptr(idx),
                                  _ptr(cand), _ptr(rend), _ptr(w), _ptr(lab), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "kmpp_seed_parallel")
    return idx, out_centers, cand, rend, w, lab, ws


def kmpp_seed_parallel_workspace_bytes(N: int, d: int, K: int, rounds: int, ell: float) -> int:
    return int(lib().kmpp_seed_parallel_workspace_bytes(N, d, K, rounds, ell))


# ---------------------------------------------------------------- Lloyd
def kmpp_lloyd_workspace_bytes(N: int, d: int, K: int, dtype: int = KMPP_F32) -> int:
    return int(lib().kmpp_lloyd_workspace_bytes(N, d, K, dtype))


def kmpp_lloyd(X: torch.Tensor, C: torch.Tensor, iters: int, *, X_exp=None, dtype: int = KMPP_F32,
               out_labels=None, out_cost=None, out_changed=None, out_counts=None, ws=None, stream=None):
    """`iters` Lloyd iterations from the centres C (FP32 [K, d], updated in
    place).  X is [N, d] in `dtype`.  Returns (C, labels int32 [N],
    cost FP64 [iters], changed int64 [iters], counts int32 [K], ws)."""
    N, d = _check_rows(X, X_exp, dtype)
    K = _centres(C, d)
    dev = X.device
    out_labels = torch.empty(N, dtype=torch.int32, device=dev) if out_labels is None else out_labels
    out_cost = torch.empty(max(iters, 1), dtype=torch.float64, device=dev) if out_cost is None else out_cost
    out_changed = torch.empty(max(iters, 1), dtype=torch.int64, device=dev) if out_changed is None else out_changed
    out_counts = torch.empty(K, dtype=torch.int32, device=dev) if out_counts is None else out_counts
    _expect(out_labels, "out_labels", dtype=torch.int32, numel=N)
    _expect(out_cost, "out_cost", dtype=torch.float64, min_numel=iters)
    _expect(out_changed, "out_changed", dtype=torch.int64, min_numel=iters)
    _expect(out_counts, "out_counts", dtype=torch.int32, numel=K)
    _require_cuda(X, C, X_exp, out_labels, out_cost, out_changed, out_counts, ws)
    if ws is None:
        ws = workspace(kmpp_lloyd_workspace_bytes(N, d, K, dtype), dev)
    rc = lib().kmpp_lloyd(_ptr(X), _ptr(X_exp), dtype, N, d, K, _ptr(C), iters, _ptr(out_labels), _ptr(out_cost),
                          _ptr(out_changed), _ptr(out_counts), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "kmpp_lloyd")
    return C, out_labels, out_cost[:iters], out_changed[:iters], out_counts, ws


# ---------------------------------------------------------------- batched
def _instances(Xs, Ks, outs, dtype=KMPP_F32, Xqs=None, Xq_exps=None):
    if len(Xs) != len(Ks) or len(Xs) != len(outs):
        raise ValueError("one K and one output triple per instance")
    _check_dtype(dtype)
    if dtype != KMPP_F32 and (Xqs is None or len(Xqs) != len(Xs)):
        raise ValueError("BF16 / FP8 batches need one stored-row tensor per instance (Xq)")
    if dtype == KMPP_FP8_E4M3 and (Xq_exps is None or len(Xq_exps) != len(Xs)):
        raise ValueError("FP8 batches need one row-exponent tensor per instance (Xq_exp)")
    arr = (Instance * len(Xs))()
    for b, (X, K, (C, D, I)) in enumerate(zip(Xs, Ks, outs)):
        N, d = _rows(X, f"Xs[{b}]")
        _expect(X, f"Xs[{b}]", dtype=torch.float32)
        _expect(C, f"outs[{b}][0]", dtype=torch.float32, numel=K * d, required=False)
        _expect(D, f"outs[{b}][1]", dtype=torch.float32, numel=N, required=False)
        _expect(I, f"outs[{b}][2]", dtype=torch.int64, numel=K, required=False)
        q = e = None
        if dtype != KMPP_F32:
            q = Xqs[b]
            e = Xq_exps[b] if dtype == KMPP_FP8_E4M3 else None
            if _check_rows(q, e, dtype, f"Xq[{b}]") != (N, d):
                raise ValueError(f"Xq[{b}] must have the shape of Xs[{b}]")
        arr[b] = Instance(X.data_ptr(), X.shape[0], X.shape[1], K, None if C is None else C.data_ptr(),
                          None if D is None else D.data_ptr(), None if I is None else I.data_ptr(),
                          dtype, None if q is None else q.data_ptr(), None if e is None else e.data_ptr())
    return arr


def kmpp_batched_workspace_bytes(Xs, Ks, *, dtype=KMPP_F32, Xq=None, Xq_exp=None) -> int:
    outs = [(None, None, None) for _ in Xs]  # output pointers are not read for sizing
    return int(lib().kmpp_batched_workspace_bytes(_instances(Xs, Ks, outs, dtype, Xq, Xq_exp), len(Xs)))


def kmpp_seed_batched_prepare(Xs, Ks, seed: int = 0, *, dtype=KMPP_F32, Xq=None, Xq_exp=None, outs=None, ws=None,
                              stream=None):
    """Plan and upload a batch.  Returns (outs, ws) with outs[b] = (centers, D, idx).
    dtype, Xq (list of stored rows, kmpp_quantize) and Xq_exp (FP8 row
    exponents) choose the rows the passes stream; one dtype per batch."""
    if len(Xs) < 1:
        raise ValueError("at least one instance")
    dev = Xs[0].device
    if outs is None:
        outs = [(torch.empty((K, X.shape[1]), dtype=torch.float32, device=dev),
                 torch.empty(X.shape[0], dtype=torch.float32, device=dev),
                 torch.empty(K, dtype=torch.int64, device=dev)) for X, K in zip(Xs, Ks)]
    arr = _instances(Xs, Ks, outs, dtype, Xq, Xq_exp)
    _require_cuda(*Xs)
    if Xq is not None:
        _require_cuda(*Xq)
    if Xq_exp is not None:
        _require_cuda(*Xq_exp)
    for o in outs:
        _require_cuda(*o)
    if ws is None:
        ws = workspace(lib().kmpp_batched_workspace_bytes(arr, len(Xs)), dev)
    _check(lib().kmpp_seed_batched_prepare(arr, len(Xs), seed, _ptr(ws), ws.numel(), _stream(stream)),
           "kmpp_seed_batched_prepare")
    return outs, ws


def kmpp_seed_batched_launch(ws: torch.Tensor, stream=None):
    _check(lib().kmpp_seed_batched_launch(_ptr(ws), _stream(stream)), "kmpp_seed_batched_launch")


def kmpp_seed_batched(Xs, Ks, seed: int = 0, *, dtype=KMPP_F32, Xq=None, Xq_exp=None, outs=None, ws=None,
                      stream=None):
    outs, ws = kmpp_seed_batched_prepare(Xs, Ks, seed, dtype=dtype, Xq=Xq, Xq_exp=Xq_exp, outs=outs, ws=ws,
                                         stream=stream)
    kmpp_seed_batched_launch(ws, stream=stream)
    return outs, ws


# ---------------------------------------------------------------- graphs
class Graph:
    """Capture what the calls inside ``with g.capture():`` enqueue on the
    current stream into a HIP graph; ``g.launch()`` replays it."""

    def __init__(self):
        self.h = ctypes.c_void_p(None)

    def capture(self, stream=None):
        g = self

        class _Ctx:
            def __enter__(self_):
                _check(lib().kmpp_graph_begin(_stream(stream)), "kmpp_graph_begin")

            def __exit__(self_, *exc):
                _check(lib().kmpp_graph_end(_stream(stream), ctypes.byref(g.h)), "kmpp_graph_end")
                return False
        return _Ctx()

    def launch(self, stream=None):
        _check(lib().kmpp_graph_launch(self.h, _stream(stream)), "kmpp_graph_launch")

    def __del__(self):
        if self.h and _lib is not None:
            _lib.kmpp_graph_destroy(self.h)
            self.h = ctypes.c_void_p(None)


def kmpp_tune_load(path: str) -> int:
    return _check(lib().kmpp_tune_load(path.encode()), "kmpp_tune_load")


def kmpp_version() -> int:
    return int(lib().kmpp_version())


def kmpp_read_probe(buf: torch.Tensor, blocks: int = 4096, nontemporal: bool = False, out=None, stream=None):
    """Read-bandwidth probe (measurement helper): reads every byte of `buf`
    once and returns the FP32 per-workgroup sums [blocks]."""
    out = torch.empty(blocks, dtype=torch.float32, device=buf.device) if out is None else out
    _expect(out, "out", dtype=torch.float32, min_numel=blocks)
    _require_cuda(buf, out)
    _check(lib().kmpp_read_probe(_ptr(buf), buf.numel() * buf.element_size(), blocks, int(nontemporal), _ptr(out),
                                 _stream(stream)), "kmpp_read_probe")
    return out
