"""Benchmark of the FP64 tiled Cholesky hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--n 32768] [--T 1024]
                    [--sched fork_join|async_dag] [--no-cpu-baseline]
    python bench.py --sweep [--ns 8192,16384,32768] [--Ts 128,256,512,1024]
                            [--scheds fork_join,async_dag,fork_join_naive,task_sync]
                            [--noop]

A step is one pass of the whole hot path over one resident synthetic input:
chol_factor (tiled right-looking factorization: every POTRF, TRSM, SYRK and
GEMM tile operation and the schedule that orders them) followed by
chol_solve of one right-hand side with the factor.  The input is the
squared-exponential kernel matrix on n points uniform in [0,1]^2
(lengthscale 0.1, nugget 1e-2), generated on the device; every step gets its
own pre-built copy, so the timed region holds nothing but the hot path.
value = (n^3/3) / mean step time, in TFLOP/s.

The default run prints one JSON line (the contract line) with
  roofline      the dominant kernel's algorithmic FP64 rate against the
                MI355X FP64 matrix peak; the kernel's launch times come from
                HIP events the library records on its own stream around each
                launch during the timed steps (chol_timing_enable);
  cpu_baseline  the CPU oracle timed on this host on a bounded sample.
  mixed         time to a solution of backward error <= 1e-12 for 16
                right-hand sides with FP32 and BF16 trailing products
                (chol_factor_mixed + chol_solve_refine) against the plain
                FP64 factor + solve, on the same matrix.
  batched       4096 SPD matrices G G^T / n + I with orders log-uniform in
                [32, 2048] (seed 3), each factored and solved for one
                right-hand side: one persistent launch
                (chol_factor_solve_batched, tuned tile sides) against a
                loop of chol_factor + chol_solve per matrix.
--serve runs the serving comparison: Poisson arrivals of factor + solve
requests (SE kernel on n points, n log-uniform in [64, 8192], lengthscale
U[0.05, 0.5], nugget 1e-2, 1-8 right-hand sides, tolerance 1e-6 or 1e-12)
at each rate, served with continuous batching (chol_server, one tick =
one batched launch) and by the one-at-a-time FP64 baseline; one JSON line
per (rate, server) with solves/s and p50/p99 latency.
--mixed prints only that comparison, one JSON line per precision;
--batched likewise for the batched comparison.
--sweep prints one JSON line per (n, T, schedule) with factor-only times
(3 warm-ups, then the median of --reps runs with min and max); those lines
are not the contract line.  Schedules: fork_join (collapsed), async_dag,
fork_join_naive and task_sync (the paper's other two variants).  With
--noop the schedules run with empty unit bodies and the lines give the
schedule's own cost per work unit (the per-task overhead of Results,
"Problem Size Scaling").
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Cholesky TFLOP/s (n^3/3) & served solves/s + p99 at bwd err<=1e-12"
FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak (published)
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}  # dense matrix peaks (published)

# HBM traffic of the trailing-update kernel per launch, from two rocprofv3
# --pmc passes (FETCH_SIZE, WRITE_SIZE) over the default configuration, each
# scaled by what the same counter reads for a plain copy of known size
# (fetch x2.0, write x1.0).  `sources` is the SHA-256 of the kernel's device
# code (KERNEL_SOURCES) the counters were taken with: if it differs, the
# figure no longer describes this kernel and the line reports traffic as null.
TRAFFIC = {
    # (schedule, n, T): (bytes per launch of the roofline kernel, sha256 of the
    # kernel sources); the profiles under profiles/ hold the counter readings
    # (forkjoin_n32768_T1024_kernels.md, lookahead_n32768_T1024_kernels.md)
    ("fork_join", 32768, 1024): (14691539678,
                                 "d285ac6b36ad61e52db4c46962ddea1ee97ebb3f000c665c0fc2dbd841f6e989"),
    # lookahead: the bulk of one step (its pool launch and tail summed)
    ("fork_join_lookahead", 32768, 1024): (12910698553,
                                           "fced0e1f0915ab1cf65b20f775ecc1d5b85f7826684ae574dff6cbfa456fb38d"),
}
# the device code the counters describe: the tile bodies, the DAG decode, the
# fork-join kernels (unit runners up to the naive variant) of kernels.hip,
# and for the lookahead schedule its split-update kernel
KERNEL_SOURCES = [("paper_2606_11937_amd/csrc/tile_ops.h", None, None),
                  ("paper_2606_11937_amd/csrc/dag.h", None, None),
                  ("paper_2606_11937_amd/csrc/kernels.hip",
                   "// ------------------------------------------------------------ unit runners",
                   "// Naive fork-join")]
KERNEL_SOURCES_EXTRA = {
    "fork_join_lookahead": [("paper_2606_11937_amd/csrc/kernels.hip",
                             "// ------------------------------------------------- fork-join with lookahead",
                             "// ----------------------------------------------- low-precision trailing update")],
}


def sources_sha(sched: str = "fork_join") -> str:
    h = hashlib.sha256()
    for path, start, end in KERNEL_SOURCES + KERNEL_SOURCES_EXTRA.get(sched, []):
        with open(os.path.join(ROOT, path), "rb") as f:
            text = f.read()
        if start is not None:
            i = text.index(start.encode())
            text = text[i:text.index(end.encode(), i)]
        h.update(text)
    return h.hexdigest()


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=32768)
    p.add_argument("--T", type=int, default=1024)
    p.add_argument("--sched", default="fork_join_lookahead",
                   choices=["async_dag", "fork_join", "fork_join_naive", "task_sync", "fork_join_lookahead"])
    p.add_argument("--nrhs", type=int, default=1)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=4096, help="order of the oracle's leading-block sample")
    p.add_argument("--sweep", action="store_true")
    p.add_argument("--ns", default="8192,16384,32768")
    p.add_argument("--Ts", default="128,256,512,1024")
    p.add_argument("--scheds", default="fork_join,async_dag")
    p.add_argument("--reps", type=int, default=20)
    p.add_argument("--noop", action="store_true", help="sweep with empty unit bodies (schedule overhead)")
    p.add_argument("--Ms", default=None, help="fixed tile counts per dimension: T = ceil(n / M) (overrides --Ts)")
    p.add_argument("--lookaheads", default=None,
                   help="async ticket-order ablation: bulk units per chain link, e.g. -1,0,1000000000")
    p.add_argument("--mixed", action="store_true",
                   help="only the mixed-precision comparison (time to a 1e-12 solution, 16 right-hand sides)")
    p.add_argument("--no-mixed", action="store_true", help="leave the mixed-precision comparison out")
    p.add_argument("--mixed-T", type=int, default=512,
                   help="tile side of the mixed-precision factorizations (the mixed workload's T=512)")
    p.add_argument("--mixed-T2", type=int, default=1024,
                   help="a second tile side for the mixed comparison in the contract line (0: none)")
    p.add_argument("--batched", action="store_true",
                   help="only the batched comparison (4096 orders log-uniform in [32, 2048], one launch vs a loop)")
    p.add_argument("--no-batched", action="store_true", help="leave the batched comparison out")
    p.add_argument("--batch-count", type=int, default=4096)
    p.add_argument("--serve", action="store_true",
                   help="only the serving comparison (Poisson arrivals, continuous batching vs one at a time)")
    p.add_argument("--rates", default="100,200,500,1000,2000,5000")
    p.add_argument("--serve-seconds", type=float, default=2.0,
                   help="arrivals per rate: min(2000, rate x this many seconds)")
    p.add_argument("--serve-resident", type=float, default=0.3,
                   help="--serve: also a stream where this fraction of arrivals are solves against resident factors")
    p.add_argument("--no-serve", action="store_true", help="leave the serving figures out of the contract line")
    p.add_argument("--serve-plans", default=None,
                   help="measure serving precision plans: 'loose,strict;...' (FP32 from these orders on)")
    p.add_argument("--batch-lookaheads", default="-1",
                   help="batched ticket order: bulk units per chain link of each matrix (comma list; -1 default)")
    return p.parse_args()


def make_input(n: int):
    from paper_2606_11937_amd import inputs
    return inputs.se_kernel_device(n, seed=1, device="cuda")


def update_flops(n: int, T: int, beyond_next: bool = False) -> float:
    """Algorithmic flops of all SYRK + GEMM tile operations (T^3 per SYRK,
    2 T^3 per GEMM, on the tiles' actual sides when T does not divide n).
    beyond_next: only the output tiles (I, K) with K > J + 1 of each step J,
    the part the lookahead schedule runs on its second stream."""
    M = -(-n // T)
    side = [min(T, n - I * T) for I in range(M)]
    f = 0.0
    for J in range(M):
        t = side[J]
        k0 = J + 2 if beyond_next else J + 1
        for I in range(k0, M):
            f += side[I] * side[I] * t  # SYRK(I, J)
            for K in range(k0, I):
                f += 2.0 * side[I] * side[K] * t  # GEMM(I, K, J)
    return f


def time_factor(tc, A0, T, sched, reps, warm=3, noop=False):
    """Median / min / max device time (ms) of chol_factor on fresh copies."""
    import torch
    n = A0.shape[0]
    A = torch.empty_like(A0)
    work = tc.factor_workspace(n, T, sched)
    st = torch.cuda.current_stream()
    times = []
    for r in range(reps + warm):
        A.copy_(A0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        tc.chol_factor(A, T, sched, work=work, stream=st, sync=False, noop=noop)
        e1.record(st)
        torch.cuda.synchronize()
        info = tc.chol_factor_info(work, st)
        if info != 0:
            raise RuntimeError(f"factor failed: info={info} (n={n} T={T} {sched})")
        if r >= warm:
            times.append(e0.elapsed_time(e1))
    del A
    return statistics.median(times), min(times), max(times)


def sweep(args):
    import torch
    from paper_2606_11937_amd import tilechol as tc
    for n in [int(x) for x in args.ns.split(",")]:
        A0 = make_input(n)
        torch.cuda.synchronize()
        Ts = [-(-n // int(M)) for M in args.Ms.split(",")] if args.Ms else [int(x) for x in args.Ts.split(",")]
        looks = [int(x) for x in args.lookaheads.split(",")] if args.lookaheads else [None]
        for T, sched, look in [(T, s, l) for T in Ts for s in args.scheds.split(",") for l in looks]:
            if look is not None:
                tc.chol_set_lookahead(look)
            med, lo, hi = time_factor(tc, A0, T, sched, args.reps, noop=args.noop)
            if look is not None:
                tc.chol_set_lookahead(-1)
            line = {"kind": "sweep", "n": n, "T": T, "M": -(-n // T), "sched": sched, "reps": args.reps,
                    "ms_median": round(med, 3), "ms_min": round(lo, 3), "ms_max": round(hi, 3)}
            if look is not None:
                line["lookahead"] = look
            if args.noop:
                units = tc.chol_dag_counts(n, T)["units"]
                line.update({"noop": True, "units": units, "us_per_unit": round(med * 1e3 / units, 4)})
            else:
                tf = n ** 3 / 3 / (med * 1e-3) / 1e12
                line.update({"tflops": round(tf, 2), "frac_fp64_peak": round(tf / FP64_MFMA_PEAK_TFLOPS, 4)})
            print(json.dumps(line), flush=True)
        del A0
        torch.cuda.empty_cache()


def cpu_model() -> str:
    """Host CPU model name (from /proc/cpuinfo, else the platform string)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(block, m: int):
    """The CPU oracle (right-looking FP64, OpenMP over the host threads it is
    given) on the leading m x m principal block of the same input (copied
    before any factor ran).  `cores` is the thread count the oracle ran with;
    the host's CPUs available to this process and their model are recorded
    beside it."""
    import oracle
    a = block.numpy()
    t0 = time.perf_counter()
    _, info = oracle.potrf(a)
    dt = time.perf_counter() - t0
    assert info == 0
    return {"value": round(m ** 3 / 3 / dt / 1e12, 6), "unit": "TFLOP/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": round(dt, 2),
            "host_cpus_available": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
            "omp": {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OMP_PROC_BIND", "OMP_PLACES")},
            "sample": f"leading {m}x{m} principal block of the same SE matrix, factored by the right-looking "
                      f"FP64 oracle; rate = ({m}^3/3)/t"}


def mixed_compare(tc, A0, T64: int, T: int, nrhs: int = 16, reps: int = 3, tol: float = 1e-12):
    """Time to an FP64 solution of A X = B with backward error <= tol.

    fp64: chol_factor (fork-join, T64) + chol_solve; its backward error is
          then measured (not timed) with chol_solve_refine at max_iter = 0.
    fp32: chol_factor_mixed (FP32 trailing products, diagonal scaling) +
          iterative refinement.
    bf16: chol_factor_mixed with BF16 trailing products and the smallest
          diagonal shift of the ladder 0, 1e-3 4^k that factors, + PCG;
          the timed region holds the whole ladder: the failed attempts
          (each a factorization and a copy of A) and the successful one.
    Each line: median of `reps` runs of the whole timed region (device
    events), iterations, final backward error, forward error and row-scaled
    factor difference against the FP64 result, and the trailing-update rate
    of the mixed factorization against its precision's matrix peak."""
    import numpy as np
    import torch
    n = A0.shape[0]
    g = np.random.default_rng(2)
    B = torch.from_numpy(g.standard_normal((n, nrhs))).cuda()
    st = torch.cuda.current_stream()
    L = torch.empty_like(A0)
    X = torch.empty_like(B)
    dsq = torch.sqrt(torch.diagonal(A0)).unsqueeze(1)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    out = {}
    # ---- FP64 reference path
    w64 = tc.factor_workspace(n, T64, "fork_join")
    sw = torch.empty(max(tc.chol_solve_workspace_size(n, T64, nrhs), 8), dtype=torch.uint8, device="cuda")
    rw = torch.empty(tc.chol_refine_workspace_size(n, T64, nrhs), dtype=torch.uint8, device="cuda")
    ts = []
    for r in range(reps + 1):
        L.copy_(A0)
        X.copy_(B)
        torch.cuda.synchronize()
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(st)
        tc.chol_factor(L, T64, "fork_join", work=w64, stream=st, sync=False)
        e1.record(st)
        tc.chol_solve(L, X, T64, work=sw, stream=st)
        e2.record(st)
        torch.cuda.synchronize()
        if r:
            ts.append((e0.elapsed_time(e1), e1.elapsed_time(e2)))
    assert tc.chol_factor_info(w64, st) == 0
    L64 = torch.tril(L)
    X64 = torch.empty_like(B)
    ok, it, eta = tc.chol_solve_refine(A0, L, B, X64, T64, "ir", tol, 0, work=rw)
    tot64 = statistics.median([a + b for a, b in ts])
    out["fp64"] = {"T": T64, "factor_ms": round(statistics.median([a for a, _ in ts]), 3),
                   "solve_ms": round(statistics.median([b for _, b in ts]), 3), "total_ms": round(tot64, 3),
                   "eta": max(eta), "meets_tol": max(eta) <= tol}
    Xref = X64
    # ---- mixed paths
    for prec in ("fp32", "bf16"):
        wm = torch.empty(tc.chol_factor_mixed_workspace_size(n, T, prec), dtype=torch.uint8, device="cuda")
        rwm = torch.empty(tc.chol_refine_workspace_size(n, T, nrhs), dtype=torch.uint8, device="cuda")
        ladder = [0.0] if prec == "fp32" else [0.0] + [1e-3 * 4 ** k for k in range(8)]
        failed = []
        shift = None
        for s_try in ladder:
            L.copy_(A0)
            info = tc.chol_factor_mixed(L, T, prec, shift=s_try, work=wm, stream=st)
            if info == 0:
                shift = s_try
                break
            failed.append({"shift": s_try, "info": info})
        if shift is None:
            out[prec] = {"T": T, "failed": failed}
            continue
        method = "ir" if prec == "fp32" else "pcg"
        runs = []
        for r in range(reps + 1):
            L.copy_(A0)
            torch.cuda.synchronize()
            if r == reps:
                # the low-precision factor runs the lookahead schedule: the
                # column-(J+1) launches ("update") and the bulk pools
                # ("update_rest") never overlap each other
                tc.chol_timing_enable(["update", "update_rest"])
            e0, e1, e2 = ev(), ev(), ev()
            e0.record(st)
            # the timed region holds the whole shift ladder: every failed
            # attempt (a factorization that meets a non-positive pivot, then a
            # fresh copy of A) before the one that succeeds
            for f in failed:
                tc.chol_factor_mixed(L, T, prec, shift=f["shift"], work=wm, stream=st, sync=False)
                L.copy_(A0)
            tc.chol_factor_mixed(L, T, prec, shift=shift, work=wm, stream=st, sync=False)
            e1.record(st)
            if r == reps:
                tc.chol_timing_enable(0)
                tm = tc.chol_timing_read(st)
                upd = (tm["update"][0] + tm["update_rest"][0],)
            ok, it, eta = tc.chol_solve_refine(A0, L, B, X, T, method, tol, 200, work=rwm, stream=st)
            e2.record(st)
            torch.cuda.synchronize()
            if r and r < reps:
                runs.append((e0.elapsed_time(e1), e1.elapsed_time(e2)))
            if r == 0:
                runs_first = (e0.elapsed_time(e1), e1.elapsed_time(e2))
        if not runs:
            runs = [runs_first]
        tot = statistics.median([a + b for a, b in runs])
        erow = (torch.tril(L) - L64).abs().div(dsq).max().item()
        fe = ((X - Xref).abs().max() / Xref.abs().max()).item()
        uflops = update_flops(n, T)
        urate = uflops / (upd[0] * 1e-3) / 1e12 if upd[0] > 0 else None
        out[prec] = {"T": T, "shift": shift, "failed_shifts": failed, "method": method,
                     "factor_ms": round(statistics.median([a for a, _ in runs]), 3),
                     "refine_ms": round(statistics.median([b for _, b in runs]), 3), "total_ms": round(tot, 3),
                     "iterations": it, "converged": ok, "eta": max(eta), "forward_err_vs_fp64": fe,
                     "e_row_vs_fp64": erow, "speedup_vs_fp64": round(tot64 / tot, 3),
                     "update_tflops": round(urate, 2) if urate else None,
                     "update_frac_of_peak": round(urate / MFMA_PEAK_TFLOPS[prec], 4) if urate else None}
        del wm, rwm
    del L, X, w64, sw, rw
    torch.cuda.empty_cache()
    return out


def batched_compare(tc, count: int = 4096, seed: int = 3, reps: int = 3):
    """One persistent launch factoring and solving a whole batch against a
    loop of chol_factor (fork-join, the library's default tile for each
    order) + chol_solve per matrix, on the same inputs.  Times are device
    time between events around the whole batch (the loop's launch gaps
    count).  The roofline floor is sum_i max(flops_i / FP64 peak, bytes_i /
    HBM peak) with flops n^3/3 and bytes 8 n^2 (the lower triangle read and
    written once)."""
    import torch
    from paper_2606_11937_amd import inputs
    sizes = inputs.batch_sizes(count, seed)
    As = inputs.gg_batch_device(sizes, seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed + 1)
    Bs = [torch.randn(n, generator=g, dtype=torch.float64, device="cuda") for n in sizes]
    Ls = [A.clone() for A in As]
    Xs = [b.clone() for b in Bs]
    st = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def reset():
        for L, A in zip(Ls, As):
            L.copy_(A)
        for X, b in zip(Xs, Bs):
            X.copy_(b)
        torch.cuda.synchronize()

    work = torch.empty(tc.chol_factor_solve_batched_workspace_size(sizes), dtype=torch.uint8, device="cuda")
    one = []
    for r in range(reps + 1):
        reset()
        e0, e1 = ev(), ev()
        e0.record(st)
        tc.chol_factor_solve_batched(Ls, Xs, work=work, stream=st, sync=False)
        e1.record(st)
        torch.cuda.synchronize()
        if r:
            one.append(e0.elapsed_time(e1))
    reset()
    infos = tc.chol_factor_solve_batched(Ls, Xs, work=work, stream=st)
    worst = 0.0
    for A, x, b in zip(As, Xs, Bs):
        r_ = b - A @ x
        den = A.abs().sum(dim=1).max() * x.abs().max() + b.abs().max()
        worst = max(worst, (r_.abs().max() / den).item())
    # the loop baseline: one workspace sized for the largest order, reused
    nmax = max(sizes)
    wf = torch.empty(max(tc.chol_factor_workspace_size(nmax, tc.chol_default_tile(nmax)), 8), dtype=torch.uint8,
                     device="cuda")
    ws = torch.empty(max(tc.chol_solve_workspace_size(nmax, 128, 1), 8), dtype=torch.uint8, device="cuda")
    loop = []
    for r in range(2):
        reset()
        e0, e1 = ev(), ev()
        e0.record(st)
        for L, X, n in zip(Ls, Xs, sizes):
            T = tc.chol_default_tile(n)
            tc.chol_factor(L, T, "fork_join", work=wf, stream=st, sync=False)
            tc.chol_solve(L, X.view(n, 1), T, work=ws, stream=st)
        e1.record(st)
        torch.cuda.synchronize()
        loop.append(e0.elapsed_time(e1))
    # the FP32 variant: FP32 trailing products, the originals kept, every
    # solution refined in FP64 to eta <= 1e-12 inside the same launch
    Ls32 = [torch.empty_like(A) for A in As]
    wm = torch.empty(tc.chol_factor_solve_batched_mixed_workspace_size(sizes, None, ["fp32"] * len(sizes)),
                     dtype=torch.uint8, device="cuda")
    fp32 = []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record(st)
        tc.chol_factor_solve_batched_mixed(As, Ls32, Bs, Xs, precs=["fp32"] * len(sizes), tol=1e-12, max_iter=10,
                                           work=wm, stream=st, sync=False)
        e1.record(st)
        torch.cuda.synchronize()
        if r:
            fp32.append(e0.elapsed_time(e1))
    inf32, it32, eta32 = tc.chol_factor_solve_batched_mixed(As, Ls32, Bs, Xs, precs=["fp32"] * len(sizes),
                                                            tol=1e-12, max_iter=10, work=wm, stream=st)
    worst32 = 0.0
    for A, x, b in zip(As, Xs, Bs):
        r_ = b - A @ x
        den = A.abs().sum(dim=1).max() * x.abs().max() + b.abs().max()
        worst32 = max(worst32, (r_.abs().max() / den).item())
    del Ls32, wm
    flops = sum(n ** 3 / 3 for n in sizes)
    floor_ms = sum(max(n ** 3 / 3 / (FP64_MFMA_PEAK_TFLOPS * 1e12), 8.0 * n * n / 8e12) for n in sizes) * 1e3
    t1 = statistics.median(one)
    tl = min(loop)
    t32 = statistics.median(fp32)
    out = {"count": count, "n_min": min(sizes), "n_max": nmax, "n_median": int(statistics.median(sizes)),
           "flops": flops, "one_launch_ms": round(t1, 3), "one_launch_tflops": round(flops / (t1 * 1e-3) / 1e12, 3),
           "loop_ms": round(tl, 3), "speedup_vs_loop": round(tl / t1, 2), "floor_ms": round(floor_ms, 3),
           "frac_of_floor": round(floor_ms / t1, 4), "worst_eta": worst,
           "all_factored": all(i == 0 for i in infos),
           "fp32": {"one_launch_ms": round(t32, 3), "one_launch_tflops": round(flops / (t32 * 1e-3) / 1e12, 3),
                    "speedup_vs_fp64_launch": round(t1 / t32, 3), "speedup_vs_loop": round(tl / t32, 2),
                    "frac_of_floor": round(floor_ms / t32, 4), "worst_eta": worst32,
                    "reported_eta_max": max(eta32), "corrections_max": max(it32),
                    "corrections_mean": round(sum(it32) / len(it32), 3), "all_factored": all(i == 0 for i in inf32),
                    "what": "FP32 trailing products, originals kept, FP64 refinement to 1e-12 in the same launch"}}
    del As, Bs, Ls, Xs, work, wf, ws
    torch.cuda.empty_cache()
    return out


def serve_compare(tc, rate: float, count: int, seed: int, mode: str, arena_gb: float = 96.0,
                  resident: float = 0.0, plan=None, wait_limit_s: float = 2.0):
    """Submit `count` requests with exponential inter-arrival times (rate per
    second) to a fresh server, from this thread at their scheduled times,
    then collect every result.  Latency is the server's own: submission to
    the result in host memory.  solves/s counts requests whose backward error
    met their tolerance, over the span from the first arrival to the last
    completion.
    resident > 0: the stream also holds solves against resident factors:
    every factor + solve request asks to keep its factor, and each arrival is,
    with probability `resident`, a solve (new right-hand sides, same
    tolerance class) against the factor of a random earlier request whose
    result is already in (factors the server evicted are refused and counted).
    The server runs with a dependency-wait limit of wait_limit_s: a wait that
    runs out restarts its request once (see chol_server_wait).
    """
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    arr = np.cumsum(gaps) - gaps[0]
    reqs = []
    for _ in range(count):
        n = int(np.rint(np.exp(rng.uniform(np.log(64), np.log(8192)))))
        nrhs = int(rng.integers(1, 9))
        reqs.append((rng.random((n, 2)), rng.standard_normal((n, nrhs)), float(rng.uniform(0.05, 0.5)), 1e-2,
                     1e-6 if rng.random() < 0.5 else 1e-12))
    solve_draw = rng.random(count)
    arena = torch.empty(int(arena_gb * (1 << 30)), dtype=torch.uint8, device="cuda")
    prev = tc.chol_set_wait_limit(wait_limit_s)  # the server keeps the limit it was created with
    try:
        srv = tc.Server(arena, 8 << 30, mode)
    finally:
        tc.chol_set_wait_limit(prev)
    if plan is not None:
        srv.set_plan(*plan)
    ids, lag, kinds = [], 0.0, []
    done_factors = []  # (factor handle, n, tol) of finished keep requests
    refused = 0
    import collections
    watch = collections.deque()  # indices of keep requests not yet seen finished
    t0 = time.perf_counter()
    for k, (p, B, ell, nug, tol) in enumerate(reqs):
        target = t0 + arr[k]
        while time.perf_counter() < target:
            pass
        lag = max(lag, time.perf_counter() - target)
        if resident > 0 and solve_draw[k] < resident:
            # harvest finished keep requests without blocking (they finish
            # roughly in arrival order: stop at the first one still running)
            while watch:
                j = watch[0]
                if srv.wait(ids[j], timeout=0.0, want_x=False)[0] == tc.CHOL_ETIMEOUT:
                    break  # still running
                f = srv.request_info(ids[j])[0]
                if f >= 0:
                    done_factors.append((f, reqs[j][1].shape[0], reqs[j][4]))
                watch.popleft()
            if done_factors:
                f, n, tol0 = done_factors[int(rng.integers(len(done_factors)))]
                try:
                    ids.append(srv.submit_solve(f, rng.standard_normal((n, B.shape[1])), tol0))
                    kinds.append("solve")
                    reqs[k] = (None, np.empty((n, B.shape[1])), ell, nug, tol0)
                    continue
                except tc.TileCholError:
                    refused += 1
        ids.append(srv.submit(p, B, ell, nug, tol, keep=resident > 0))
        kinds.append("factor")
        if resident > 0:
            watch.append(len(ids) - 1)
    lat, met, worst = {1e-6: [], 1e-12: []}, 0, 0.0
    lat_solve = []
    statuses, missed, precs, corr = {}, [], {}, 0
    for rid, r, kind in zip(ids, reqs, kinds):
        st, _, eta, latency, info = srv.wait(rid, timeout=600.0, want_x=False)
        lat[r[4]].append(latency)
        if kind == "solve":
            lat_solve.append(latency)
        met += st == tc.CHOL_OK
        worst = max(worst, eta)
        statuses[str(st)] = statuses.get(str(st), 0) + 1
        _, pr, c, _ = srv.request_info(rid)
        precs[str(pr)] = precs.get(str(pr), 0) + 1
        corr += c
        if st != tc.CHOL_OK and len(missed) < 8:
            missed.append({"n": r[1].shape[0], "nrhs": r[1].shape[1], "tol": r[4], "status": st, "info": info,
                           "eta": eta, "latency_ms": round(latency * 1e3, 1)})
    t_end = time.perf_counter()
    ticks = srv.ticks()
    evictions = srv.evictions()
    srv.close()
    del arena
    torch.cuda.empty_cache()
    allv = sorted(lat[1e-6] + lat[1e-12])
    pct = lambda v, q: round(float(np.percentile(v, q)) * 1e3, 3) if v else None
    span = t_end - t0  # arrivals start at t0; the last wait returns at the last completion or later
    out = {"rate": rate, "requests": count, "server": mode, "met_tolerance": int(met),
           "solves_per_s": round(met / span, 1), "span_s": round(span, 3), "ticks": ticks,
           "p50_ms": pct(allv, 50), "p99_ms": pct(allv, 99),
           "p50_ms_tol1e-6": pct(lat[1e-6], 50), "p99_ms_tol1e-6": pct(lat[1e-6], 99),
           "p50_ms_tol1e-12": pct(lat[1e-12], 50), "p99_ms_tol1e-12": pct(lat[1e-12], 99),
           "worst_eta": worst, "max_submit_lag_ms": round(lag * 1e3, 3), "statuses": statuses,
           "precisions": precs, "corrections": corr, "missed": missed}
    if resident > 0:
        out.update({"resident_solves": len(lat_solve), "refused_evicted": refused, "evictions": evictions,
                    "p50_ms_resident_solve": pct(lat_solve, 50), "p99_ms_resident_solve": pct(lat_solve, 99)})
    return out


def serve_summary(tc, rates=(500.0, 2000.0), seconds: float = 1.0):
    """The serving figures of the contract line: for each rate, continuous
    batching and the one-at-a-time FP64 baseline on the same Poisson stream
    (min(2000, rate x seconds) requests), and at the highest rate the stream
    with solves against resident factors."""
    out = {"workload": "Poisson arrivals of factor + solve requests: SE kernel on n points uniform in [0,1]^2, "
                       "n log-uniform in [64, 8192], lengthscale U[0.05, 0.5], nugget 1e-2, 1-8 right-hand "
                       "sides, tolerance 1e-6 or 1e-12 (1/2 each); seed 4",
           "rates": []}
    for rate in rates:
        count = int(min(2000, max(50, rate * seconds)))
        row = {"rate": rate}
        for mode in ("continuous", "fifo"):
            r = serve_compare(tc, rate, count, 4, mode)
            row[mode] = {k: r[k] for k in ("requests", "met_tolerance", "solves_per_s", "p50_ms", "p99_ms",
                                          "p99_ms_tol1e-6", "p99_ms_tol1e-12", "worst_eta", "ticks",
                                          "precisions", "corrections", "statuses")}
        row["throughput_vs_fifo"] = round(row["continuous"]["solves_per_s"] / row["fifo"]["solves_per_s"], 2)
        out["rates"].append(row)
    r = serve_compare(tc, max(rates), int(min(2000, max(rates) * seconds)), 5, "continuous", resident=0.3)
    out["resident"] = {k: r[k] for k in ("rate", "requests", "met_tolerance", "solves_per_s", "p50_ms", "p99_ms",
                                         "resident_solves", "p50_ms_resident_solve", "p99_ms_resident_solve",
                                         "refused_evicted", "evictions", "worst_eta")}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is a design, "
              "not a build. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.sweep:
        return sweep(args)
    from paper_2606_11937_amd import tilechol as tc
    if args.serve_plans:
        # the precision plan's thresholds, measured: (FP32 from n, loose; strict)
        for pl in args.serve_plans.split(";"):
            plan = tuple(int(x) for x in pl.split(","))
            for rate in [float(x) for x in args.rates.split(",")]:
                count = int(min(2000, max(50, rate * args.serve_seconds)))
                r = serve_compare(tc, rate, count, 4, "continuous", plan=plan)
                print(json.dumps({"kind": "serve_plan", "plan": plan, **r}), flush=True)
        return
    if args.serve:
        for rate in [float(x) for x in args.rates.split(",")]:
            count = int(min(2000, max(50, rate * args.serve_seconds)))
            for mode in ("continuous", "fifo"):
                print(json.dumps({"kind": "serve", **serve_compare(tc, rate, count, 4, mode)}), flush=True)
            if args.serve_resident > 0:
                r = serve_compare(tc, rate, count, 5, "continuous", resident=args.serve_resident)
                print(json.dumps({"kind": "serve_resident", **r}), flush=True)
        return
    if args.batched:
        for la in [int(x) for x in args.batch_lookaheads.split(",")]:
            tc.chol_set_lookahead(la)
            print(json.dumps({"kind": "batched", "lookahead": la, **batched_compare(tc, args.batch_count)}),
                  flush=True)
        tc.chol_set_lookahead(-1)
        return
    if args.mixed:
        A0 = make_input(args.n)
        res = mixed_compare(tc, A0, args.T, args.mixed_T)
        for prec, r in res.items():
            print(json.dumps({"kind": "mixed", "n": args.n, "nrhs": 16, "prec": prec, **r}), flush=True)
        return

    n, T, sched, K, W = args.n, args.T, args.sched, args.steps, args.warmup
    print(f"[bench] n={n} T={T} sched={sched} steps={K} warmup={W}", file=sys.stderr, flush=True)
    A0 = make_input(n)
    sample = None if args.no_cpu_baseline else A0[:args.cpu_sample, :args.cpu_sample].cpu()
    copies = [A0.clone() for _ in range(K + W)]  # A0 stays pristine for the comparisons below
    g = torch.Generator(device="cpu").manual_seed(2)
    rhs = [torch.randn(n, args.nrhs, generator=g, dtype=torch.float64).cuda() for _ in range(K + W)]
    works = [tc.factor_workspace(n, T, sched) for _ in range(K + W)]
    nb = tc.chol_solve_workspace_size(n, T, args.nrhs)
    swork = torch.empty(max(nb, 8), dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def step(i, ev=None):
        if ev is not None:
            ev[0].record(st)
        tc.chol_factor(copies[i], T, sched, work=works[i], stream=st, sync=False)
        if ev is not None:
            ev[1].record(st)
        tc.chol_solve(copies[i], rhs[i], T, work=swork, stream=st)

    for i in range(W):
        step(i)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tc.chol_timing_read(st)  # discard anything recorded before
    # time the dominant kernel's launches only: every event pair costs a few
    # microseconds on the stream
    tc.chol_timing_enable(["update_rest"] if sched == "fork_join_lookahead" else
                          ["update"] if sched.startswith("fork_join") else ["persistent"])
    torch.cuda.synchronize()
    t_start.record(st)
    for k in range(K):
        step(W + k, evs[k])
    t_end.record(st)
    torch.cuda.synchronize()
    tc.chol_timing_enable(0)
    launches = tc.chol_timing_read(st)
    total_ms = t_start.elapsed_time(t_end)
    factor_ms = [a.elapsed_time(b) for a, b in evs]
    print(f"[bench] timed {K} steps: {total_ms:.2f} ms; factor ms {['%.2f' % x for x in factor_ms]}",
          file=sys.stderr, flush=True)
    for i in range(K + W):
        info = tc.chol_factor_info(works[i], st)
        if info != 0:
            raise RuntimeError(f"factor {i} failed with info={info}")
    ms_step = total_ms / K
    flops = n ** 3 / 3
    value = flops / (ms_step * 1e-3) / 1e12

    if sched == "fork_join_lookahead":
        # the bulk of each step's update: one interval per step (its pool
        # launch on the second stream and that launch's tail on the caller's
        # stream share one unit counter), one step at a time, so the summed
        # intervals fit inside the step
        kernel = ("tc_fj_update_pool (SYRK+GEMM trailing update of the tile columns beyond J+1: per step a launch on "
                  "the second stream leaving workgroup slots to the next panel chain, and a tail launch on the "
                  "caller's stream behind that chain, on one unit counter; timed from the first's start to the "
                  "later end)")
        kms, kcount = launches["update_rest"]
        kflops = update_flops(n, T, beyond_next=True) * K
    elif sched.startswith("fork_join"):
        kernel = {"fork_join": "tc_fj_update (collapsed SYRK+GEMM trailing update, one launch per step)",
                  "fork_join_naive": "tc_fj_update_naive (trailing update parallel over tile rows, one launch per step)",
                  }[sched]
        kms, kcount = launches["update"]
        kflops = update_flops(n, T) * K  # over the K timed factorizations
    elif sched == "task_sync":
        kernel = "tc_sync (persistent kernel with grid barriers, one launch per factorization)"
        kms, kcount = launches["persistent"]
        kflops = flops * K
    else:
        kernel = "tc_async (persistent DAG kernel, one launch per factorization)"
        kms, kcount = launches["persistent"]
        kflops = flops * K
    avg_launch_ms = kms / max(kcount, 1)
    flops_per_launch = kflops / max(kcount, 1)
    achieved = flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
    traffic = None
    rec = TRAFFIC.get((sched, n, T))
    if rec is not None and rec[1] == sources_sha(sched):
        traffic = rec[0]
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"FP64 tiled Cholesky factor + {args.nrhs}-RHS solve of the SE-kernel SPD matrix "
                               f"(n={n}, points uniform in [0,1]^2, lengthscale 0.1, nugget 1e-2), tile T={T}, "
                               f"{sched} schedule",
                   "n": n, "T": T, "schedule": sched, "nrhs": args.nrhs},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4), "traffic": traffic,
                     "kernel": kernel, "launches": kcount, "flops_per_launch": flops_per_launch,
                     "avg_launch_ms": round(avg_launch_ms, 4),
                     # the kernel's summed launch time per step, inside ms_per_step
                     "kernel_ms_per_step": round(kms / K, 3),
                     "step_frac": round(value / FP64_MFMA_PEAK_TFLOPS, 4)},
        "factor_ms": {"median": round(statistics.median(factor_ms), 3), "min": round(min(factor_ms), 3),
                      "max": round(max(factor_ms), 3)},
        "factor_tflops_median": round(flops / (statistics.median(factor_ms) * 1e-3) / 1e12, 3),
        "launch_ms_per_factor": {k: [round(v[0] / K, 3), v[1] // K] for k, v in launches.items() if v[1]},
    }
    del copies, works, rhs
    torch.cuda.empty_cache()
    if not args.no_mixed:
        print("[bench] mixed-precision comparison", file=sys.stderr, flush=True)
        out["mixed"] = mixed_compare(tc, A0, T, args.mixed_T)
        if args.mixed_T2 and args.mixed_T2 != args.mixed_T:
            out[f"mixed_T{args.mixed_T2}"] = mixed_compare(tc, A0, T, args.mixed_T2)
    del A0
    torch.cuda.empty_cache()
    if not args.no_batched:
        print("[bench] batched comparison", file=sys.stderr, flush=True)
        out["batched"] = batched_compare(tc, args.batch_count)
    if not args.no_serve:
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serve"] = serve_summary(tc)
    if sample is not None:
        print(f"[bench] cpu baseline on a {args.cpu_sample}^2 sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sample, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
