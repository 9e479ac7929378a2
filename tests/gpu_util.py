"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the FP64 oracle under the stated tolerances.

Tolerances (FP32 distances, FP64 sums):
  * D: |D_gpu - D_or| <= 1e-5 * D_or elementwise (D_or == 0 => D_gpu == 0);
  * seeds: the first seed exactly; every later draw either equal to the
    oracle's draw on the D built from the GPU's earlier seeds (replay), or
    t = u * sum(D) within 1e-6 * sum(D) of a CDF boundary and inside the GPU
    index's oracle interval up to that tolerance;
  * centres: bit-identical copies of the chosen original rows.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle

D_RTOL = 1e-5
T_TOL = 1e-6


def check_D(D_gpu: np.ndarray, D_or: np.ndarray, rtol: float = D_RTOL):
    D_gpu = D_gpu.astype(np.float64)
    zero = D_or == 0.0
    assert np.all(D_gpu[zero] == 0.0), f"{int((D_gpu[zero] != 0).sum())} rows with oracle D == 0 are nonzero"
    err = np.abs(D_gpu - D_or)
    bad = err > rtol * D_or
    assert not bad.any(), (f"{int(bad.sum())} D values outside {rtol} relative; worst rel "
                           f"{float((err[~zero] / D_or[~zero]).max()):.3e}")


def check_seed_run(X: np.ndarray, K: int, seed: int, idx: np.ndarray, centers: np.ndarray, D: np.ndarray,
                   Xd: np.ndarray | None = None, zero_seed_rows: bool = False, inst: int = 0,
                   exact: bool = False):
    """Replay the oracle on the GPU's seeds and apply the parity rules.
    Returns the oracle result and the number of draws that differed (accepted
    near a boundary)."""
    Xd = X if Xd is None else Xd
    r = oracle.seed(Xd, K, seed=seed, inst=inst, Xc=X, zero_seed_rows=zero_seed_rows, replay=idx)
    assert r.status >= 0, r.status
    assert int(idx[0]) == int(r.idx[0]), "first seed differs"
    differ = 0
    for m in range(1, K):
        g = int(idx[m])
        if g != int(r.idx[m]):
            assert not exact, f"draw {m}: gpu {g} oracle {int(r.idx[m])}"
            assert oracle.seed_index_ok(g, r.rec[m], int(r.idx[m]), T_TOL), \
                f"draw {m}: gpu {g} oracle {int(r.idx[m])} rec {r.rec[m].tolist()}"
            differ += 1
    np.testing.assert_array_equal(centers, X[idx])
    if exact:
        np.testing.assert_array_equal(D.astype(np.float64), r.D)
    else:
        check_D(D, r.D)
    return r, differ


def run_seed(lib, X: torch.Tensor, K: int, seed: int = 0, **kw):
    idx, C, D, ws = lib.kmpp_seed(X, K, seed, **kw)
    st = lib.kmpp_status(ws)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), C.cpu().numpy(), D.cpu().numpy(), st
