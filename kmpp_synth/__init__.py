"""Seeded synthetic inputs for k-means++ seeding.

This module only draws data: it holds none of the seeding or assignment
arithmetic, so both the FP64 oracle's tests and the HIP path's tests and
benchmark can take their inputs from here without sharing method code.

The paper measures on 2-D points whose distribution it does not state
(Section III); these Gaussian / Student-t mixtures stand in for its
workloads and for the five named workload shapes:

  ``small``     N=10,000, d=2, K=16: 16 isotropic Gaussians, sigma=1, means
                uniform in [-10,10]^2, exactly 625 points each, rows shuffled
  ``plain``     N=1,000,000, d=32, K=256: 256 Gaussians, means uniform in
                [-50,50]^32, per-component sigma uniform in [0.5,2],
                Dirichlet(1) weights, multinomial component counts
  ``unitsphere`` N=4,194,304, d=128, K=1024: 1024 random unit means, point =
                normalize(mean + 0.1 * N(0, I)), uniform component choice
  ``batched``   512 instances: N log-uniform in [1e3, 2e5], d in {8,16,64},
                K uniform in [8,256]; each a K-component mixture, sigma=1,
                means uniform in [-20,20]^d, uniform component choice
  ``large``     N=16,777,216, d=64, K=4096: 4096 components, means uniform in
                [-100,100]^64, Student-t (nu=3) noise of scale 1
  ``paper_k`` / ``paper_n``  the paper's own shapes (N=4M, d=2, K=100 and
                N=10M, d=2, K=50) as isotropic mixtures, sigma=1, means
                uniform in [-100,100]^2

Every draw comes from a ``torch.Generator`` seeded with a fixed integer per
workload (and per instance for the batched form), on the requested device;
rows are generated in 2^20-row chunks to bound temporaries.  The same seed
on the same device type gives the same tensor.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

CHUNK = 1 << 20


@dataclass
class Workload:
    name: str
    N: int
    d: int
    K: int
    X: torch.Tensor                       # FP32 [N, d] row-major
    labels: torch.Tensor | None = None    # generating component per row
    means: torch.Tensor | None = None
    meta: dict = field(default_factory=dict)


def _gen(device, seed: int) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _uniform(shape, lo, hi, g, device):
    return torch.rand(shape, generator=g, device=device, dtype=torch.float64) * (hi - lo) + lo


def _shuffled_equal_labels(N, K, g, device):
    lab = torch.arange(N, device=device) % K
    perm = torch.randperm(N, generator=g, device=device)
    return lab[perm]


def _rows(N, d, labels, means, noise_fn, device):
    X = torch.empty((N, d), dtype=torch.float32, device=device)
    for a in range(0, N, CHUNK):
        b = min(N, a + CHUNK)
        lab = labels[a:b]
        X[a:b] = (means[lab] + noise_fn(b - a, lab)).to(torch.float32)
    return X


def small(device="cpu", seed: int = 0) -> Workload:
    N, d, K = 10_000, 2, 16
    g = _gen(device, 1000 + seed)
    means = _uniform((K, d), -10.0, 10.0, g, device)
    labels = _shuffled_equal_labels(N, K, g, device)
    X = _rows(N, d, labels, means,
              lambda n, lab: torch.randn((n, d), generator=g, device=device, dtype=torch.float64), device)
    return Workload("small", N, d, K, X, labels, means)


def plain(device="cpu", seed: int = 0, N: int = 1_000_000, d: int = 32, K: int = 256) -> Workload:
    g = _gen(device, 2000 + seed)
    means = _uniform((K, d), -50.0, 50.0, g, device)
    sig = _uniform((K,), 0.5, 2.0, g, device)
    w = -torch.log(torch.rand((K,), generator=g, device=device, dtype=torch.float64).clamp_min(1e-300))
    w = w / w.sum()                                   # Dirichlet(1) = normalised Exp(1)
    labels = torch.multinomial(w.float(), N, replacement=True, generator=g)
    X = _rows(N, d, labels, means,
              lambda n, lab: sig[lab][:, None] * torch.randn((n, d), generator=g, device=device,
                                                             dtype=torch.float64), device)
    return Workload("plain", N, d, K, X, labels, means, {"sigma": sig, "weights": w})


def unitsphere(device="cpu", seed: int = 0, N: int = 4_194_304, d: int = 128, K: int = 1024) -> Workload:
    g = _gen(device, 3000 + seed)
    m = torch.randn((K, d), generator=g, device=device, dtype=torch.float64)
    means = m / m.norm(dim=1, keepdim=True)
    labels = torch.randint(0, K, (N,), generator=g, device=device)
    X = torch.empty((N, d), dtype=torch.float32, device=device)
    for a in range(0, N, CHUNK):
        b = min(N, a + CHUNK)
        v = means[labels[a:b]] + 0.1 * torch.randn((b - a, d), generator=g, device=device, dtype=torch.float64)
        X[a:b] = (v / v.norm(dim=1, keepdim=True)).to(torch.float32)
    return Workload("unitsphere", N, d, K, X, labels, means)


def large(device="cpu", seed: int = 0, N: int = 16_777_216, d: int = 64, K: int = 4096) -> Workload:
    g = _gen(device, 5000 + seed)
    means = _uniform((K, d), -100.0, 100.0, g, device).to(torch.float32)
    labels = torch.randint(0, K, (N,), generator=g, device=device)

    def t3(n, lab):
        z = torch.randn((n, d), generator=g, device=device)
        v = torch.randn((3, n, d), generator=g, device=device).square_().sum(0)
        return z * torch.rsqrt(v / 3.0)

    X = torch.empty((N, d), dtype=torch.float32, device=device)
    for a in range(0, N, CHUNK):
        b = min(N, a + CHUNK)
        X[a:b] = means[labels[a:b]] + t3(b - a, None)
    return Workload("large", N, d, K, X, labels, means)


def paper_shape(which: str, device="cpu", seed: int = 0) -> Workload:
    N, K = (4_000_000, 100) if which == "paper_k" else (10_000_000, 50)
    d = 2
    g = _gen(device, 6000 + seed + (0 if which == "paper_k" else 1))
    means = _uniform((K, d), -100.0, 100.0, g, device)
    labels = torch.randint(0, K, (N,), generator=g, device=device)
    X = _rows(N, d, labels, means,
              lambda n, lab: torch.randn((n, d), generator=g, device=device, dtype=torch.float64), device)
    return Workload(which, N, d, K, X, labels, means)


@dataclass
class BatchSpec:
    N: list
    d: list
    K: list


def batched_spec(n_inst: int = 512, seed: int = 0, n_lo: int = 1_000, n_hi: int = 200_000,
                 dims=(8, 16, 64), k_lo: int = 8, k_hi: int = 256) -> BatchSpec:
    """Shapes of the batched workload: N log-uniform in [n_lo, n_hi], d uniform
    over ``dims``, K uniform in [k_lo, k_hi] (K <= N always holds)."""
    g = _gen("cpu", 4000 + seed)
    u = torch.rand((n_inst,), generator=g, dtype=torch.float64)
    Ns = torch.round(torch.exp(math.log(n_lo) + u * (math.log(n_hi) - math.log(n_lo)))).long().tolist()
    ds = [dims[i] for i in torch.randint(0, len(dims), (n_inst,), generator=g).tolist()]
    Ks = torch.randint(k_lo, k_hi + 1, (n_inst,), generator=g).tolist()
    Ks = [min(k, n) for k, n in zip(Ks, Ns)]
    return BatchSpec(Ns, ds, Ks)


def batched_instance(b: int, N: int, d: int, K: int, device="cpu", seed: int = 0) -> torch.Tensor:
    g = _gen(device, 40_000 + 1000 * seed + b)
    means = _uniform((K, d), -20.0, 20.0, g, device)
    labels = torch.randint(0, K, (N,), generator=g, device=device)
    return _rows(N, d, labels, means,
                 lambda n, lab: torch.randn((n, d), generator=g, device=device, dtype=torch.float64), device)


def lattice(N: int, d: int, lim: int = 100, device="cpu", seed: int = 0) -> torch.Tensor:
    """Integer coordinates in [-lim, lim]: every squared distance is an integer
    below 2^24 for lim=100, d<=8, so FP32 distances are exact."""
    g = _gen(device, 7000 + seed)
    return torch.randint(-lim, lim + 1, (N, d), generator=g, device=device).to(torch.float32)


def gaussian(N: int, d: int, device="cpu", seed: int = 0, scale: float = 1.0) -> torch.Tensor:
    g = _gen(device, 8000 + seed)
    return (scale * torch.randn((N, d), generator=g, device=device)).contiguous()


def workload(name: str, device="cpu", seed: int = 0) -> Workload:
    return {"small": small, "plain": plain, "unitsphere": unitsphere, "large": large}[name](device=device,
                                                                                          seed=seed)
