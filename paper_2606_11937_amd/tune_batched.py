"""Offline autotuner of the batched factorization's tile side.

    python -m paper_2606_11937_amd.tune_batched [--out gpurun_out/batched_tiles.json]

For every n-bucket a batch of orders drawn log-uniformly inside the bucket
(G G^T / n + I matrices, one right-hand side each) is factored and solved by
chol_factor_solve_batched with each candidate tile side given explicitly;
the fastest side (median of 3 runs) becomes the bucket's row of the table.
The table is chosen from (n, precision) only, and the library compiles it in
(build.py turns the JSON into tc_tuned_batched_tile and
tc_tuned_batched_tile_fp32).  --prec fp64 (the default) sweeps
chol_factor_solve_batched and writes the "fp64" table; --prec fp32 sweeps
chol_factor_solve_batched_mixed with every matrix in FP32 (refined to 1e-12)
and writes the "fp32" table.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

BUCKETS = [(32, 128), (129, 256), (257, 512), (513, 1024), (1025, 2048), (2049, 4096)]
CANDIDATES = [0, 64, 128, 256, 512, 1024]  # 0: one tile (T = n)


def main():
    import torch
    from paper_2606_11937_amd import inputs, tilechol as tc
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning", "batched_tiles.json"))
    ap.add_argument("--flops", type=float, default=3e11, help="work per bucket batch (n^3/3 summed)")
    ap.add_argument("--prec", choices=["fp64", "fp32"], default="fp64")
    args = ap.parse_args()
    fp32 = args.prec == "fp32"
    rows = []
    log = []
    for lo, hi in BUCKETS:
        # orders drawn in the bucket until the batch holds `flops` of work
        # (at least 16 and at most 2048 matrices)
        pool = inputs.batch_sizes(2048, seed=11, lo=lo, hi=hi)
        sizes, acc = [], 0.0
        for n in pool:
            if len(sizes) >= 16 and acc >= args.flops:
                break
            sizes.append(n)
            acc += n ** 3 / 3
        count = len(sizes)
        As = inputs.gg_batch_device(sizes, seed=11)
        g = torch.Generator(device="cuda")
        g.manual_seed(12)
        Bs = [torch.randn(n, generator=g, dtype=torch.float64, device="cuda") for n in sizes]
        Ls = [A.clone() for A in As]
        Xs = [b.clone() for b in Bs]
        best = None
        for T in CANDIDATES:
            if T == 0 and hi > 256:
                continue  # one tile per matrix only for small orders
            if T != 0 and T >= hi:
                continue
            Ts = [n if T == 0 else T for n in sizes]
            if fp32:
                precs = ["fp32"] * count
                wbytes = tc.chol_factor_solve_batched_mixed_workspace_size(sizes, Ts, precs)
            else:
                wbytes = tc.chol_factor_solve_batched_workspace_size(sizes, Ts)
            work = torch.empty(wbytes, dtype=torch.uint8, device="cuda")
            times = []
            for r in range(4):
                if not fp32:  # the FP32 path reads the originals and writes L and x itself
                    for L, A in zip(Ls, As):
                        L.copy_(A)
                    for X, b in zip(Xs, Bs):
                        X.copy_(b)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                if fp32:
                    tc.chol_factor_solve_batched_mixed(As, Ls, Bs, Xs, Ts=Ts, precs=precs, work=work, sync=False)
                else:
                    tc.chol_factor_solve_batched(Ls, Xs, Ts, work=work, sync=False)
                e1.record()
                torch.cuda.synchronize()
                if r:
                    times.append(e0.elapsed_time(e1))
            ms = statistics.median(times)
            flops = sum(n ** 3 / 3 for n in sizes)
            rec = {"prec": args.prec, "bucket": [lo, hi], "count": count, "T": T, "ms": round(ms, 3),
                   "tflops": round(flops / (ms * 1e-3) / 1e12, 2)}
            print(json.dumps(rec), flush=True)
            log.append(rec)
            if best is None or ms < best[1]:
                best = (T, ms)
        rows.append({"n_max": hi, "T": best[0]})
        del As, Bs, Ls, Xs
        torch.cuda.empty_cache()
    rows.append({"n_max": 1048576, "T": 1024})
    # the file's other tables (the other precision's tile table, the serving
    # plan) are kept as they are
    out = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            out = json.load(f)
    out.update({
        "about": ("Tile side T of each matrix of a batched factorization, chosen from (n, precision) only. Rows "
                  "are n-buckets: a matrix of order n takes the first row with n <= n_max; T = 0 means one tile "
                  "(T = n). Written by paper_2606_11937_amd/tune_batched.py from a sweep on MI355X."),
        "source": "measured: median of 3 batched factor+solve runs per (bucket, T) on one MI355X",
        args.prec: rows,
        "sweep" if not fp32 else "sweep_fp32": log,
    })
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"table": rows}), flush=True)


if __name__ == "__main__":
    main()
