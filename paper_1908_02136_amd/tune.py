"""Autotuner for libkmpp's launch schedules (run on the GPU).

* Seed pass: for each (storage format, d) it times whole seeding runs over a
  grid of (threads per workgroup, rows per tile, row loads in flight per
  lane, cached or non-temporal row loads) and keeps the fastest;
* batched planner: it times the 512-instance batch over a grid of the
  cost-model knobs (workgroups per CU, the cap on one instance's time) and
  keeps the fastest.

The result is written as text lines
``seed <dtype> <d> <threads> <rows> <loads per lane> <non-temporal>`` and
``batched <key> <value>`` to ``tune_table.txt`` next to the library, which
the binding loads at import (``kmpp_tune_load``).

    python -m paper_1908_02136_amd.tune [--quick] [--out PATH]
"""
from __future__ import annotations

import argparse
import os
import sys

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _time(fn, reps=2):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_seed(kl, cases, quick):
    lines = []
    for dtype, d, N, K in cases:
        X = torch.randn((N, d), device="cuda")
        Xq = E = None
        if dtype:
            Xq, E = kl.kmpp_quantize(X, dtype)
        row_bytes = d * {0: 4, 1: 2, 2: 1}[dtype]
        rpt_grid = sorted({max(1, (b // row_bytes)) for b in ([32 << 10, 64 << 10, 128 << 10, 256 << 10]
                                                                if not quick else [64 << 10, 128 << 10])})
        best = None
        for nt in (256, 512):
            for rpt in rpt_grid:
                for u in (8, 16):
                    for ntl in (0, 1):
                        try:
                            ms = _time(lambda: kl.kmpp_seed(X, K, 0, Xq=Xq, Xq_exp=E, dtype=dtype, threads=nt,
                                                            rows_per_tile=rpt, loads_per_lane=u, row_loads=ntl))
                        except kl.KmppError:
                            continue
                        print(f"seed dtype={dtype} d={d} N={N} K={K} threads={nt} rows={rpt} u={u} nt={ntl}: "
                              f"{ms:.3f} ms", flush=True)
                        if best is None or ms < best[0]:
                            best = (ms, nt, rpt, u, ntl)
        if best:
            lines.append(f"seed {dtype} {d} {best[1]} {best[2]} {best[3]} {best[4]}")
        del X, Xq, E
        torch.cuda.empty_cache()
    return lines


def tune_batched(kl, quick):
    import kmpp_synth
    spec = kmpp_synth.batched_spec()
    Xs = [kmpp_synth.batched_instance(b, spec.N[b], spec.d[b], spec.K[b], device="cuda") for b in range(512)]
    best = None
    path = os.path.join(HERE, "_tune_tmp.txt")
    for wpc in (1, 2):
        for alpha in ((0.5, 1.0, 2.0) if not quick else (1.0,)):
            with open(path, "w") as f:
                f.write(f"batched wg_per_cu {wpc}\nbatched alpha {alpha}\n")
            kl.kmpp_tune_load(path)
            outs, ws = kl.kmpp_seed_batched_prepare(Xs, spec.K, 0)
            ms = _time(lambda: kl.kmpp_seed_batched_launch(ws), reps=2)
            st = kl.kmpp_status(ws)
            print(f"batched wg_per_cu={wpc} alpha={alpha}: {ms:.2f} ms status {st}", flush=True)
            if st == 0 and (best is None or ms < best[0]):
                best = (ms, wpc, alpha)
    os.remove(path)
    if best is None:
        return []
    return [f"batched wg_per_cu {best[1]}", f"batched alpha {best[2]}"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=os.path.join(HERE, "tune_table.txt"))
    args = ap.parse_args()
    import paper_1908_02136_amd as kl
    kl.lib()
    cases = [  # (dtype, d, N, K): the shapes the benchmark runs
        (0, 32, 1_000_000, 256), (0, 128, 4_194_304, 64), (1, 128, 4_194_304, 64), (2, 128, 4_194_304, 64),
        (0, 64, 16_777_216, 16), (1, 64, 16_777_216, 16), (2, 64, 16_777_216, 16), (0, 2, 10_000, 16),
        (0, 8, 200_000, 64), (0, 16, 200_000, 64),
    ]
    lines = ["# written by paper_1908_02136_amd/tune.py on " + torch.cuda.get_device_name(0)]
    lines += tune_seed(kl, cases, args.quick)
    lines += tune_batched(kl, args.quick)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
