"""Toy-size FP64 k-means++ in NumPy / pure Python -- TEST INFRASTRUCTURE ONLY.

A second, independent write-up of the oracle (paper, Section II,
Algorithm 1) used to cross-check ``kmpp_oracle.c`` on small inputs.  It
recomputes every point's distance to *all* chosen seeds at each step, the
way the paper's per-thread design does (Section II: each thread handles one
point against every selected centroid), instead of keeping D incrementally,
so a mistake in the incremental update of the C oracle cannot hide here.
"""
from __future__ import annotations

import math

import numpy as np

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11) in Python integers."""
    x0, x1, x2, x3 = (int(v) & _MASK for v in ctr)
    k0, k1 = (int(v) & _MASK for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        pa = _M0 * x0
        pb = _M1 * x2
        x0, x1, x2, x3 = ((pb >> 32) ^ x1 ^ k0) & _MASK, pb & _MASK, ((pa >> 32) ^ x3 ^ k1) & _MASK, pa & _MASK
    return (x0, x1, x2, x3)


def uniform(seed: int, step: int, inst: int = 0) -> float:
    r = philox4x32_10((step, inst, 0, 0), (seed & _MASK, (seed >> 32) & _MASK))
    m = ((r[0] >> 5) << 26) | (r[1] >> 6)
    return m / float(1 << 53)


def seed(X, K: int, seed: int = 0, inst: int = 0, zero_seed_rows: bool = False):
    """Returns (indices list, final D float64 [N])."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    u0 = uniform(seed, 0, inst)
    idx = [min(int(math.floor(u0 * N)), N - 1)]
    for m in range(1, K + 1):
        C = X[idx]                                    # all chosen seeds
        d2 = ((X[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
        D = d2.min(axis=1)
        if zero_seed_rows:
            D[idx] = 0.0
        if m == K:
            return idx, D
        S = np.cumsum(D)                              # index order, FP64
        T = float(S[-1])
        u = uniform(seed, m, inst)
        if T == 0.0:
            i = min(int(math.floor(u * N)), N - 1)
        else:
            t = u * T
            i = int(np.searchsorted(S, t, side="right"))
            if i >= N:
                i = int(np.nonzero(D > 0)[0][-1])
        idx.append(i)
    raise AssertionError("unreachable")
