"""Drive the nearest-seed assignment for counter collection.

    python3 -m paper_1908_02136_amd.prof_assign CASE

CASE is one of plain-f32 (1,000,000 x 32, K = 256), unitsphere-bf16 and
unitsphere-f32 (4,194,304 x 128, K = 1024): N(0, 1) rows, the first K rows
as centres, three `kmpp_assign` calls after one untimed call.
"""
import sys

import torch

import paper_1908_02136_amd as kl

CASES = {
    "plain-f32": (1_000_000, 32, 256, kl.KMPP_F32),
    "unitsphere-bf16": (4_194_304, 128, 1024, kl.KMPP_BF16),
    "unitsphere-f32": (4_194_304, 128, 1024, kl.KMPP_F32),
}


def main(case: str) -> None:
    N, d, K, dt = CASES[case]
    g = torch.Generator(device="cuda").manual_seed(1)
    X = torch.randn((N, d), device="cuda", generator=g)
    C = X[:K].contiguous()
    Xq, E = (X, None) if dt == kl.KMPP_F32 else kl.kmpp_quantize(X, dt)
    kl.kmpp_assign(Xq, C, X_exp=E, dtype=dt)
    for _ in range(3):
        kl.kmpp_assign(Xq, C, X_exp=E, dtype=dt)
    torch.cuda.synchronize()
    print("done", case, flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "unitsphere-bf16")
