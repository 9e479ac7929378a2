"""FP64 CPU oracle for k-means++ seeding (D^2 sampling) and nearest-seed
assignment -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import this package.  The product library never
loads it and shares no code with it.

Two independent implementations live here:

* ``kmpp_oracle.c`` (wrapped below): plain FP64 C with OpenMP over points,
  used for everything above toy sizes and for the timed CPU baseline;
* ``tiny.py``: NumPy/pure-Python FP64 version for toy inputs, used to
  cross-check the C code.

Both follow the paper's Algorithm 1 ("Serial K-means++", Section II): a
uniform first seed, then each seed drawn with probability proportional to
the squared distance to the nearest chosen seed, with the sum over points in
double precision (Section II, the reduction paragraph).  Readings where the
paper is silent are stated in ``kmpp_oracle.c``'s header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kmpp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libkmpp_oracle.so")

OK = 0
W_DEGENERATE = 1
E_INVALID = -1
E_NONFINITE = -4

# per-step record layout written by kmo_seed (8 doubles per step)
REC_T, REC_t, REC_SI_LO, REC_SI_HI, REC_SG_LO, REC_SG_HI, REC_DG, REC_U = range(8)


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``oracle/libkmpp_oracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared",
               "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, u64, u32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32
        L.kmo_philox4x32_10.argtypes = [P, P, P]
        L.kmo_philox4x32_10.restype = None
        L.kmo_uniform.argtypes = [u64, u32, u32]
        L.kmo_uniform.restype = ctypes.c_double
        L.kmo_upper_bound.argtypes = [P, i64, ctypes.c_double]
        L.kmo_upper_bound.restype = i64
        L.kmo_seed.argtypes = [P, P, i64, i32, i32, u64, u32, i32, P, P, P, P, i32]
        L.kmo_seed.restype = ctypes.c_int
        L.kmo_seed_range.argtypes = [P, P, i64, i32, i32, u64, u32, i32, P, i32, i32, P, P, P, i32]
        L.kmo_seed_range.restype = ctypes.c_int
        L.kmo_draw.argtypes = [P, i64, ctypes.c_double, P, P, i32]
        L.kmo_draw.restype = ctypes.c_int
        L.kmo_wdraw.argtypes = [P, i64, ctypes.c_double, P, P]
        L.kmo_wdraw.restype = ctypes.c_int
        L.kmo_assign.argtypes = [P, i64, i32, P, i32, P, P, P, i32]
        L.kmo_assign.restype = ctypes.c_int
        L.kmo_assign_rows.argtypes = [P, i32, P, i64, P, i32, P, P, P]
        L.kmo_assign_rows.restype = ctypes.c_int
        L.kmo_pair_dist.argtypes = [P, i32, P, i64, P, P, P]
        L.kmo_pair_dist.restype = ctypes.c_int
        L.kmo_bf16_encode_n.argtypes = [P, i64, P]
        L.kmo_bf16_decode_n.argtypes = [P, i64, P]
        L.kmo_fp8_decode.argtypes = [ctypes.c_uint8]
        L.kmo_fp8_decode.restype = ctypes.c_double
        L.kmo_fp8_encode.argtypes = [ctypes.c_double]
        L.kmo_fp8_encode.restype = ctypes.c_uint8
        L.kmo_fp8_row_exponent.argtypes = [P, i32]
        L.kmo_fp8_row_exponent.restype = i32
        L.kmo_fp8_quantize_rows.argtypes = [P, i64, i32, P, P]
        L.kmo_fp8_dequantize_rows.argtypes = [P, P, i64, i32, P]
        L.kmo_fp8_quantize_rows_fast.argtypes = [P, i64, i32, P, P, i32]
        L.kmo_lloyd_update.argtypes = [P, i64, i32, P, i32, P, P, P]
        L.kmo_lloyd_update.restype = ctypes.c_int
        L.kmo_lloyd.argtypes = [P, i64, i32, i32, P, i32, P, P, P, i32]
        L.kmo_lloyd.restype = ctypes.c_int
        L.kmo_uniform4.argtypes = [u64, u32, u32, u32, u32]
        L.kmo_uniform4.restype = ctypes.c_double
        L.kmo_kmpar.argtypes = [P, i64, i32, i32, u64, u32, i32, ctypes.c_double, i64, P, P, P, P, P, P, P, P, P,
                                P, P, P, P, i32]
        L.kmo_kmpar.restype = ctypes.c_int
        L.kmo_fp8_encode_bisect.argtypes = [ctypes.c_double]
        L.kmo_fp8_encode_bisect.restype = ctypes.c_uint8
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


# ---------------------------------------------------------------- Philox
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().kmo_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed: int, step: int, inst: int = 0) -> float:
    return lib().kmo_uniform(seed, step, inst)


def upper_bound(S: np.ndarray, t: float) -> int:
    S = np.ascontiguousarray(S, dtype=np.float64)
    return lib().kmo_upper_bound(_ptr(S), S.size, t)


# ---------------------------------------------------------------- seeding
class SeedResult:
    def __init__(self, idx, D, rec, status):
        self.idx = idx          # int64 [K] oracle's own draws
        self.D = D              # float64 [N] final nearest squared distance
        self.rec = rec          # float64 [K, 8] per-step record (row 0 unused)
        self.status = status    # 0, W_DEGENERATE or negative error

    @property
    def phi(self) -> float:
        return float(np.sum(self.D))


def seed(X, K: int, seed: int = 0, inst: int = 0, Xc=None, zero_seed_rows: bool = False,
         replay=None, nthreads: int = 0, chunk: int = 0, progress=None) -> SeedResult:
    """k-means++ seeding in FP64 (Algorithm 1).  ``X`` holds the values
    distances use; ``Xc`` (default ``X``) the values centres take.  With
    ``replay`` (the GPU's indices) each step is checked on the D built from
    the replayed seeds.  ``chunk`` > 0 runs the passes in ranges of that many
    (the same arithmetic) and calls ``progress(m)`` after each range."""
    Xd = _f32(X)
    N, d = Xd.shape
    Xc_ = Xd if Xc is None else _f32(Xc)
    assert Xc_.shape == Xd.shape
    idx = np.zeros(K, dtype=np.int64)
    D = np.zeros(N, dtype=np.float64)
    rec = np.zeros((K, 8), dtype=np.float64)
    rp = None
    if replay is not None:
        rp = np.ascontiguousarray(np.asarray(replay, dtype=np.int64))
        assert rp.size == K
    if chunk <= 0:
        st = lib().kmo_seed(_ptr(Xd), _ptr(Xc_), N, d, K, seed, inst, int(zero_seed_rows),
                            _ptr(rp), _ptr(idx), _ptr(D), _ptr(rec), nthreads)
    else:
        st = OK
        for m0 in range(1, K + 1, chunk):
            m1 = min(K, m0 + chunk - 1)
            s1 = lib().kmo_seed_range(_ptr(Xd), _ptr(Xc_), N, d, K, seed, inst, int(zero_seed_rows), _ptr(rp),
                                      m0, m1, _ptr(idx), _ptr(D), _ptr(rec), nthreads)
            if s1 < 0:
                st = s1
                break
            if s1 == W_DEGENERATE:
                st = W_DEGENERATE
            if progress is not None:
                progress(m1)
    if st == E_INVALID:
        raise ValueError("oracle: invalid arguments")
    return SeedResult(idx, D, rec, st)


def draw(D, u: float, nthreads: int = 0):
    """One inverse-CDF draw of Algorithm 1 on a given D with a given u:
    returns (index or -1, status, rec4 = (T, t, S_{i-1}, S_i))."""
    D = np.ascontiguousarray(np.asarray(D, dtype=np.float64))
    out = np.zeros(1, dtype=np.int64)
    rec = np.zeros(4, dtype=np.float64)
    st = lib().kmo_draw(_ptr(D), D.size, float(u), _ptr(out), _ptr(rec), nthreads)
    if st == E_INVALID:
        raise ValueError("oracle: invalid arguments")
    return int(out[0]), st, rec


def wdraw(share, u: float):
    """One draw of the weighted k-means|| recluster on given shares (w or
    w * D) with a given u: returns (index or -1, status, rec4)."""
    sh = np.ascontiguousarray(np.asarray(share, dtype=np.float64))
    out = np.zeros(1, dtype=np.int64)
    rec = np.zeros(4, dtype=np.float64)
    st = lib().kmo_wdraw(_ptr(sh), sh.size, float(u), _ptr(out), _ptr(rec))
    if st == E_INVALID:
        raise ValueError("oracle: invalid arguments")
    return int(out[0]), st, rec


def assign(X, C, nthreads: int = 0):
    """FP64 brute-force nearest centre (ties -> smallest index).  Returns
    (labels int32 [N], min distance float64 [N], second-smallest float64 [N])."""
    X = _f32(X)
    C = _f32(C)
    N, d = X.shape
    K = C.shape[0]
    lab = np.zeros(N, dtype=np.int32)
    mind = np.zeros(N, dtype=np.float64)
    sec = np.zeros(N, dtype=np.float64)
    lib().kmo_assign(_ptr(X), N, d, _ptr(C), K, _ptr(lab), _ptr(mind), _ptr(sec), nthreads)
    return lab, mind, sec


def assign_rows(X, rows, C):
    X = _f32(X)
    C = _f32(C)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    n = rows.size
    lab = np.zeros(n, dtype=np.int32)
    mind = np.zeros(n, dtype=np.float64)
    sec = np.zeros(n, dtype=np.float64)
    lib().kmo_assign_rows(_ptr(X), X.shape[1], _ptr(rows), n, _ptr(C), C.shape[0], _ptr(lab),
                          _ptr(mind), _ptr(sec))
    return lab, mind, sec


def pair_dist(X, rows, C, cols) -> np.ndarray:
    X = _f32(X)
    C = _f32(C)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    cols = np.ascontiguousarray(np.asarray(cols, dtype=np.int32))
    out = np.zeros(rows.size, dtype=np.float64)
    lib().kmo_pair_dist(_ptr(X), X.shape[1], _ptr(rows), rows.size, _ptr(C), _ptr(cols), _ptr(out))
    return out


# ---------------------------------------------------------------- Lloyd
def lloyd_update(X, labels, C_prev):
    """One centre update: the FP64 mean of every cluster's points in index
    order, rounded to FP32; empty clusters keep their centre.  Returns
    (C float32 [K, d], counts int64 [K])."""
    X = _f32(X)
    C_prev = _f32(C_prev)
    K, d = C_prev.shape
    lab = np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
    C = np.zeros((K, d), dtype=np.float32)
    n = np.zeros(K, dtype=np.int64)
    st = lib().kmo_lloyd_update(_ptr(X), X.shape[0], d, _ptr(lab), K, _ptr(C_prev), _ptr(C), _ptr(n))
    if st != OK:
        raise ValueError("oracle: invalid arguments")
    return C, n


def lloyd(X, C0, iters: int, nthreads: int = 0):
    """`iters` Lloyd iterations from centres C0.  Returns (C after the last
    update, labels of the last assignment, cost [iters], changed [iters])."""
    X = _f32(X)
    C = _f32(C0).copy()
    N, d = X.shape
    K = C.shape[0]
    lab = np.zeros(N, dtype=np.int32)
    cost = np.zeros(iters, dtype=np.float64)
    ch = np.zeros(iters, dtype=np.int64)
    st = lib().kmo_lloyd(_ptr(X), N, d, K, _ptr(C), iters, _ptr(lab), _ptr(cost), _ptr(ch), nthreads)
    if st != OK:
        raise ValueError("oracle: invalid arguments")
    return C, lab, cost, ch


# ---------------------------------------------------------------- k-means||
def uniform4(seed: int, c0: int, c1: int, c2: int, c3: int) -> float:
    """u in [0,1) from the Philox words of counter (c0, c1, c2, c3)."""
    return lib().kmo_uniform4(seed, c0, c1, c2, c3)


class KmparResult:
    pass


def kmpar(X, K: int, seed: int = 0, rounds: int = 5, ell: float | None = None, inst: int = 0,
          cap: int | None = None, keep_D: bool = False, replay_cand=None, replay_end=None, replay_w=None,
          replay_idx=None, nthreads: int = 0) -> KmparResult:
    """k-means|| (Bahmani et al., Algorithm 2) in FP64: candidates, weights,
    labels, and the K centres of the weighted k-means++ recluster."""
    X = _f32(X)
    N, d = X.shape
    ell = float(2 * K) if ell is None else float(ell)
    cap = N if cap is None else int(cap)
    r = KmparResult()
    r.cand = np.zeros(cap, dtype=np.int64)
    nc = np.zeros(1, dtype=np.int64)
    r.round_end = np.zeros(rounds + 1, dtype=np.int64)
    r.weights = np.zeros(cap, dtype=np.int64)
    r.labels = np.zeros(N, dtype=np.int32)
    r.idx = np.zeros(K, dtype=np.int64)
    r.rec = np.zeros((K, 8), dtype=np.float64)
    r.phi = np.zeros(max(rounds, 1), dtype=np.float64)
    r.Dr = np.zeros((max(rounds, 1), N), dtype=np.float64) if keep_D else None
    conv = lambda a: None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    rc, re, rw, ri = conv(replay_cand), conv(replay_end), conv(replay_w), conv(replay_idx)
    st = lib().kmo_kmpar(_ptr(X), N, d, K, seed, inst, rounds, ell, cap, _ptr(r.cand), _ptr(nc), _ptr(r.round_end),
                         _ptr(r.weights), _ptr(r.labels), _ptr(r.idx), _ptr(r.rec), _ptr(r.phi), _ptr(r.Dr),
                         _ptr(rc), _ptr(re), _ptr(rw), _ptr(ri), nthreads)
    if st == E_INVALID:
        raise ValueError("oracle: invalid arguments or candidate capacity exceeded")
    r.status = st
    r.ncand = int(nc[0])
    r.cand = r.cand[:r.ncand]
    mc = int(re[rounds]) if re is not None else r.ncand
    r.weights = r.weights[:mc]
    return r


# ---------------------------------------------------------------- formats
def bf16_encode(x) -> np.ndarray:
    x = _f32(x)
    out = np.zeros(x.shape, dtype=np.uint16)
    lib().kmo_bf16_encode_n(_ptr(x), x.size, _ptr(out))
    return out


def bf16_decode(h) -> np.ndarray:
    h = np.ascontiguousarray(np.asarray(h, dtype=np.uint16))
    out = np.zeros(h.shape, dtype=np.float32)
    lib().kmo_bf16_decode_n(_ptr(h), h.size, _ptr(out))
    return out


def fp8_decode(q: int) -> float:
    return lib().kmo_fp8_decode(int(q))


def fp8_encode(v: float) -> int:
    return int(lib().kmo_fp8_encode(float(v)))


def fp8_row_exponent(row) -> int:
    r = _f32(row)
    return int(lib().kmo_fp8_row_exponent(_ptr(r), r.size))


def fp8_quantize_rows(X):
    X = _f32(X)
    N, d = X.shape
    q = np.zeros((N, d), dtype=np.uint8)
    e = np.zeros(N, dtype=np.int8)
    lib().kmo_fp8_quantize_rows(_ptr(X), N, d, _ptr(q), _ptr(e))
    return q, e


def fp8_encode_bisect(v: float) -> int:
    return int(lib().kmo_fp8_encode_bisect(float(v)))


def fp8_quantize_rows_fast(X, nthreads: int = 0):
    """fp8_quantize_rows with the bisection encoder, rows in parallel."""
    X = _f32(X)
    N, d = X.shape
    q = np.zeros((N, d), dtype=np.uint8)
    e = np.zeros(N, dtype=np.int8)
    lib().kmo_fp8_quantize_rows_fast(_ptr(X), N, d, _ptr(q), _ptr(e), nthreads)
    return q, e


def fp8_dequantize_rows(q, e) -> np.ndarray:
    q = np.ascontiguousarray(np.asarray(q, dtype=np.uint8))
    e = np.ascontiguousarray(np.asarray(e, dtype=np.int8))
    N, d = q.shape
    out = np.zeros((N, d), dtype=np.float32)
    lib().kmo_fp8_dequantize_rows(_ptr(q), _ptr(e), N, d, _ptr(out))
    return out


# ---------------------------------------------------------------- parity rules
def seed_index_ok(g: int, rec_row: np.ndarray, own: int, tol: float = 1e-6) -> bool:
    """Acceptance rule for one draw (replay mode): the GPU's index equals the
    oracle's, or the draw t = u * T lies within tol*T of a CDF boundary and
    inside the GPU index's oracle interval [S_{g-1}, S_g) up to tol*T, with a
    positive oracle D at g."""
    if g == own:
        return True
    T, t = rec_row[REC_T], rec_row[REC_t]
    lo_i, hi_i = rec_row[REC_SI_LO], rec_row[REC_SI_HI]
    lo_g, hi_g, dg = rec_row[REC_SG_LO], rec_row[REC_SG_HI], rec_row[REC_DG]
    eps = tol * T
    near = min(t - lo_i, hi_i - t) <= eps
    inside = (lo_g - eps <= t) and (t < hi_g + eps)
    return bool(near and inside and dg > 0)
