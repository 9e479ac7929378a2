"""Autotuner for libkmpp's launch schedules (run on the GPU).

* Seed pass: for each (storage format, d) it times whole seeding runs over a
  grid of (threads per workgroup, rows per tile, row loads in flight per
  lane, cached or non-temporal row loads, draw at the start of the next pass,
  in a draw kernel or by the next pass's first workgroup for all) and keeps
  the fastest;
* batched planner: it times the 512-instance batch over a grid of the
  cost-model knobs (workgroups per CU, the cap on one instance's time) and
  keeps the fastest.

The result is written as text lines
``seed <dtype> <d> <threads> <rows> <loads per lane> <non-temporal> <draw>``
(draw: 1 at the start of the next pass, 2 draw kernel, 3 workgroup 0 of the
next pass for all) and ``batched <key> <value>`` to
``tune_table.txt`` next to the library, which the binding loads at import
(``kmpp_tune_load``).

    python -m paper_1908_02136_amd.tune [--quick] [--out PATH]
        [--only DTYPE:D,...]   retune these cases, keep the table's other lines
        [--draw-only]          keep every schedule, re-time only the draw
        [--batched-only]       retune the batched planner, keep the seed lines
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


# the draw at pass start applies up to this many tiles (every workgroup reads
# every tile sum)
DRAW_AT_START_TILES = 2048


def tune_draw(kl, X, K, Xq, E, dtype, nt, rpt, u, ntl):
    """Fastest draw placement (KMPP_DRAW_PASS, KMPP_DRAW_KERNEL or KMPP_DRAW_LEAD) for one schedule."""
    ms = {}
    for draw in (kl.KMPP_DRAW_PASS, kl.KMPP_DRAW_KERNEL, kl.KMPP_DRAW_LEAD):
        ms[draw] = _time(lambda: kl.kmpp_seed(X, K, 0, Xq=Xq, Xq_exp=E, dtype=dtype, threads=nt, rows_per_tile=rpt,
                                              loads_per_lane=u, row_loads=ntl, draw=draw), reps=3)
        print(f"seed dtype={dtype} d={X.shape[1]} N={X.shape[0]} K={K} threads={nt} rows={rpt} u={u} nt={ntl} "
              f"draw={draw}: {ms[draw]:.3f} ms", flush=True)
    return min(ms, key=ms.get)


def _case_rows(kl, dtype, d, N):
    X = torch.randn((N, d), device="cuda")
    Xq = E = None
    if dtype:
        Xq, E = kl.kmpp_quantize(X, dtype)
    return X, Xq, E


def tune_seed(kl, cases, quick, keep=None):
    """Seed lines for `cases`; `keep` maps (dtype, d) to an existing line's
    schedule (threads, rows, u, non-temporal) to re-time only the draw."""
    lines = []
    for dtype, d, N, K in cases:
        X, Xq, E = _case_rows(kl, dtype, d, N)
        if keep is not None and (dtype, d) in keep:
            nt, rpt, u, ntl = keep[(dtype, d)]
            draw = tune_draw(kl, X, K, Xq, E, dtype, nt, rpt, u, ntl)
            lines.append(f"seed {dtype} {d} {nt} {rpt} {u} {ntl} {draw}")
            del X, Xq, E
            torch.cuda.empty_cache()
            continue
        row_bytes = d * {0: 4, 1: 2, 2: 1}[dtype]
        # tiles of 32 KiB to 2 MiB of rows (larger tiles mean fewer workgroups
        # and tile sums: on 16.7M x 64 rows, 2 MiB tiles beat 256 KiB ones
        # by 2.8 % per seed)
        rpt_grid = sorted({max(1, (b // row_bytes)) for b in ([32 << 10, 64 << 10, 128 << 10, 256 << 10, 512 << 10,
                                                                1 << 20, 2 << 20]
                                                               if not quick else [64 << 10, 128 << 10])})
        best = None
        for nt in (256, 512):
            for rpt in rpt_grid:
                draws = [kl.KMPP_DRAW_KERNEL, kl.KMPP_DRAW_LEAD]
                if -(-N // rpt) <= DRAW_AT_START_TILES:
                    draws.append(kl.KMPP_DRAW_PASS)
                for u in (8, 16):
                    for ntl in (0, 1):
                        for draw in draws:
                            try:
                                ms = _time(lambda: kl.kmpp_seed(X, K, 0, Xq=Xq, Xq_exp=E, dtype=dtype, threads=nt,
                                                                rows_per_tile=rpt, loads_per_lane=u, row_loads=ntl,
                                                                draw=draw))
                            except kl.KmppError:
                                continue
                            print(f"seed dtype={dtype} d={d} N={N} K={K} threads={nt} rows={rpt} u={u} nt={ntl} "
                                  f"draw={draw}: {ms:.3f} ms", flush=True)
                            if best is None or ms < best[0]:
                                best = (ms, nt, rpt, u, ntl, draw)
        if best:
            lines.append(f"seed {dtype} {d} {best[1]} {best[2]} {best[3]} {best[4]} {best[5]}")
        del X, Xq, E
        torch.cuda.empty_cache()
    return lines


def tune_batched(kl, quick):
    """The planner's knobs for the 512-instance batch: workgroups per CU (the
    persistent grid), the cap on one instance's time relative to the mean
    load (sets gang sizes) and the per-seed cost of a gang's exchange (the
    cost model's gang sync), timed on the whole batch."""
    import kmpp_synth
    spec = kmpp_synth.batched_spec()
    Xs = [kmpp_synth.batched_instance(b, spec.N[b], spec.d[b], spec.K[b], device="cuda") for b in range(512)]
    best = None
    path = os.path.join(HERE, "_tune_tmp.txt")
    grid = [(w, a, sw) for w in (2, 3, 4) for a in (0.0625, 0.125, 0.25, 0.5, 1.0) for sw in (0.75, 1.5, 3.0, 6.0)]
    if quick:
        grid = [(w, 1.0, 6.0) for w in (1, 2, 3, 4)]
    for wpc, alpha, syncw in grid:
        with open(path, "w") as f:
            f.write(f"batched wg_per_cu {wpc}\nbatched alpha {alpha}\nbatched syncw_us {syncw}\n")
        kl.kmpp_tune_load(path)
        outs, ws = kl.kmpp_seed_batched_prepare(Xs, spec.K, 0)
        ms = _time(lambda: kl.kmpp_seed_batched_launch(ws), reps=2)
        st = kl.kmpp_status(ws)
        print(f"batched wg_per_cu={wpc} alpha={alpha} syncw_us={syncw}: {ms:.2f} ms status {st}", flush=True)
        if st == 0 and (best is None or ms < best[0]):
            best = (ms, wpc, alpha, syncw)
    os.remove(path)
    if best is None:
        return []
    return [f"batched wg_per_cu {best[1]}", f"batched alpha {best[2]}", f"batched syncw_us {best[3]}"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=os.path.join(HERE, "tune_table.txt"))
    ap.add_argument("--only", default="", help="comma list of DTYPE:D cases to retune")
    ap.add_argument("--draw-only", action="store_true")
    ap.add_argument("--batched-only", action="store_true", help="retune the batched planner, keep the seed lines")
    args = ap.parse_args()
    import paper_1908_02136_amd as kl
    kl.lib()
    cases = [  # (dtype, d, N, K): the shapes the benchmark runs (d = 2: the paper's point sets)
        (0, 32, 1_000_000, 256), (0, 128, 4_194_304, 64), (1, 128, 4_194_304, 64), (2, 128, 4_194_304, 64),
        (0, 64, 16_777_216, 256), (1, 64, 16_777_216, 256), (2, 64, 16_777_216, 256), (0, 2, 4_000_000, 64),
        (0, 8, 200_000, 64), (0, 16, 200_000, 64),
    ]
    old = {}  # (dtype, d) -> schedule of the current table
    other = []  # its batched lines
    if (args.only or args.draw_only) and os.path.exists(args.out):
        for ln in open(args.out):
            f = ln.split()
            if len(f) >= 7 and f[0] == "seed":
                old[(int(f[1]), int(f[2]))] = tuple(int(x) for x in f[3:7])
            elif f and f[0] == "batched":
                other.append(ln.strip())
    lines = ["# written by paper_1908_02136_amd/tune.py on " + torch.cuda.get_device_name(0)]
    if args.batched_only:
        kept = [ln.strip() for ln in open(args.out) if ln.startswith("seed ")] if os.path.exists(args.out) else []
        lines += kept + tune_batched(kl, args.quick)
    elif args.only or args.draw_only:
        only = {tuple(int(x) for x in c.split(":")) for c in args.only.split(",") if c}
        keep = {k: v for k, v in old.items() if k not in only}
        lines += tune_seed(kl, [c for c in cases if (c[0], c[1]) in only or (c[0], c[1]) in keep], args.quick,
                           keep=keep)
        lines += other
    else:
        lines += tune_seed(kl, cases, args.quick)
        lines += tune_batched(kl, args.quick)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
