#!/usr/bin/env python3
"""Throughput of the fleet-staging hot path on one MI355X.

One step = the whole hot path over one synthetic instance: the FP64 haversine
cost table, base ranking, and the Tabu search for its full iteration count.
The default workload is the largest single-GPU instance: 4,000 bases, 10,000
hospitals, 100,000 missions, 64 vehicles, range 900 km, tenure 25, 200
iterations (1.6 GB cost table).

The metric is mission x move evaluations per second: every Tabu iteration
scores K*(B-K) swap moves over M missions.  It is reported for the whole step
(cost table and ranking included in the time).  Alongside:
  roofline      the swap sweep's algorithmic bytes per launch over its average
                launch time (HIP events on its own stream), against 8 TB/s HBM;
                its counter-measured HBM traffic and VALU issue rate when the
                profiles hold them for the current kernel source;
  cpu_baseline  the CPU oracle on a bounded sample of the same search, on every
                host core and on one core, with the CPU model; the oracle runs
                on the GPU's table and its trajectory must equal the GPU's;
  dense         (sparse-sweep workloads) the same workload with the dense sweep;
  medium        the 500-base, 20,000-mission, 30-vehicle workload (500
                iterations): throughput and its sweep's roofline;
  fleet         the heterogeneous fleet (heliports, rotary-only missions,
                rotary- and fixed-wing vehicles) on the medium workload: the
                typed relocation search's solves/s and its sweep roofline;
  portfolio     the paper's permuted local and Tabu searches (random scan
                orders), ten seeds each in one batch launch: runs/s and the
                upper / lower / average result;
  optimum       a synthetic analogue of the paper's Table 1 and Fig. 2:
                eleven small datasets against their exact optimum by GPU
                enumeration (base ranking, random starts, ten-seed local and
                Tabu searches: upper / lower / average gap);
  batch         the ragged batch (1,024 instances of uneven size, 200
                iterations each): solves/s of one launch against one solve
                per instance, results identical;
  serve         the repositioning load (95% small / 5% large instances, 10% of
                the missions redrawn, 100 warm-started iterations per request):
                solves/s at saturation and p50/p99 latency under Poisson
                arrivals at 0.5/0.8/1.0x the plain path's saturation rate, for
                the plain path (one table build + one solve per request) and
                the server, whose results must be identical; then one stream
                under a 1 GB budget that forces evictions.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# int32 VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def run_workload(fs, torch, profiling, workload, steps, warmup, iterations=None, sparse=None,
                 timing_every=8):
    """Times `steps` whole steps (indexed cost table + ranking + N Tabu
    iterations) of a workload with its inputs resident.  sparse: None = the
    library's choice, 0 / 1 = force the dense / sparse sweep."""
    from paper_2001_05291_amd import synth

    c = synth.WORKLOADS[workload]
    B, M, K, R, T, N = c["B"], c["M"], c["K"], c["R"], c["T"], c["N"]
    if iterations is not None:
        N = iterations
    inst = synth.workload_instance(workload)
    dev = torch.device("cuda:0")
    bases = torch.from_numpy(inst.bases).to(dev)
    hospitals = torch.from_numpy(inst.hospitals).to(dev)
    mission_ph = torch.from_numpy(inst.mission_ph).to(dev)
    old = os.environ.get("FS_SPARSE")
    if sparse is not None:
        os.environ["FS_SPARSE"] = str(int(sparse))
    result = {}

    def step():
        # the indexed builder: missions as hospital-id pairs (the same table,
        # bitwise, as from the missions' coordinates)
        C, _ = fs.build_cost_table_indexed(bases, hospitals, mission_ph)
        r = fs.tabu_solve(C, K, R, T, N, want_assign=True, want_trace=False)
        result["r"] = r
        result["C"] = C

    try:
        for w in range(warmup):
            step()
            log(f"[bench] {workload}: warmup {w + 1}/{warmup} done")
        torch.cuda.synchronize()
        # every `timing_every`-th sweep / refresh launch carries dispatch-stamped
        # events (a dispatch with events is followed by a gap, so timing all of
        # them would slow the timed loop itself)
        fs.timing_enable(True, every=timing_every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        sweep_ms, sweep_n = fs.timing_read("sweep")
        refresh_ms, refresh_n = fs.timing_read("refresh")
        fin_ms, fin_n = fs.timing_read("finalize")
        fused_ms, fused_n = fs.timing_read("score_refresh")
        fs.timing_enable(False)
    finally:
        if sparse is not None:
            if old is None:
                os.environ.pop("FS_SPARSE", None)
            else:
                os.environ["FS_SPARSE"] = old
    log(f"[bench] {workload}: timed {steps} steps in {elapsed:.4f} s")

    evals_per_step = N * K * (B - K) * M
    # dominant kernel: the swap sweep.  Dense: every closed row once (4 B per
    # element) + the per-mission state (b1, b2, o1).  Sparse (its block
    # scoring runs as a kernel of its own, timed as "finalize", or fused with
    # the refresh, timed as "score_refresh"): the sorted-list entries the walk
    # needs at the final placement + the state once per base block.
    is_sparse = fin_n > 0 or fused_n > 0
    r = result["r"]
    if is_sparse:
        sweep_bytes = profiling.sparse_sweep_bytes(result["C"].cpu().numpy(),
                                                   r.best_open.cpu().numpy())
    else:
        sweep_bytes = (B - K) * M * 4 + 12 * M
    sweep_avg_s = (sweep_ms / max(sweep_n, 1)) / 1e3
    achieved = sweep_bytes / sweep_avg_s / 1e9 if sweep_n else None
    kname = "k_sweep_sparse" if is_sparse else "k_sweep"
    traffic = profiling.read_traffic(
        os.path.join(ROOT, "profiles", f"{kname}_{workload}_traffic.md"), workload)
    valu = profiling.read_valu(
        os.path.join(ROOT, "profiles", f"{kname}_{workload}_valu.md"), workload)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                "kernel": kname, "bytes_per_launch": sweep_bytes,
                "avg_launch_us": sweep_avg_s * 1e6, "launches": sweep_n}
    if valu is not None and sweep_n:
        # VALU lane-operations per launch (counted) over the live launch time
        rate = valu / sweep_avg_s
        roofline["valu"] = {"lane_ops_per_launch": valu, "achieved_ops_per_s": rate,
                            "peak_ops_per_s": VALU_PEAK_OPS, "frac": rate / VALU_PEAK_OPS}
    else:
        roofline["valu"] = None
    return {
        "workload": workload, "B": B, "H": c["H"], "M": M, "K": K, "R": R, "T": T, "N": N,
        "seed": c["seed"], "steps": steps, "warmup": warmup,
        "value": evals_per_step * steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
        "roofline": roofline,
        "detail": {"sweep_path": "sparse" if is_sparse else "dense",
                   "sparse_score_ms_per_launch": fin_ms / max(fin_n, 1) if fin_n else None,
                   "score_refresh_ms_per_launch": fused_ms / max(fused_n, 1) if fused_n else None,
                   "sweep_ms_per_launch": sweep_ms / max(sweep_n, 1),
                   "refresh_ms_per_launch": refresh_ms / max(refresh_n, 1),
                   "best_coverage": r.coverage, "best_distance_m": r.distance,
                   "best_iter": r.best_iter},
        "_C": result["C"], "_r": r,
    }


def cpu_baseline(fs, oracle, main, n_all, n_one):
    """The oracle's Tabu search on the GPU's table (host copy): n_all
    iterations on every host thread, n_one on one thread.  Its trajectory
    must equal the GPU's over the iterations it ran."""
    B, M, K, R, T, N = (main[k] for k in ("B", "M", "K", "R", "T", "N"))
    C = main["_C"]
    Ch = C.cpu().numpy()
    g = fs.tabu_solve(C, K, R, T, N, want_assign=False, want_trace=True)
    threads = oracle.get_threads()
    t1 = time.perf_counter()
    o = oracle.tabu(Ch, K, R, T, n_all)
    s_all = time.perf_counter() - t1
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        o1 = oracle.tabu(Ch, K, R, T, n_one)
        s_one = time.perf_counter() - t1
    finally:
        oracle.set_threads(threads)
    tr = g.trace[:n_all]
    same = all(np.array_equal(tr[f], getattr(o, f)) for f in
               ("out_base", "in_base", "moved", "cur_cov", "cur_dist", "best_cov", "best_dist"))
    same = same and all(np.array_equal(g.trace[:n_one][f], getattr(o1, f))
                        for f in ("out_base", "in_base", "cur_dist"))
    if n_all == N:
        same = same and np.array_equal(g.best_open.cpu().numpy(), o.best_open) and \
            (g.coverage, g.distance, g.best_iter) == (o.coverage, o.distance, o.best_iter)
    if not same:
        raise SystemExit("cpu baseline: the oracle's trajectory differs from the GPU's")
    per = K * (B - K) * M
    return {"value": n_all * per / s_all, "unit": "MM-evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {n_all} of {N} Tabu iterations of the same instance on the GPU's "
                      f"table, {threads} threads, {s_all:.2f} s; trajectory equal to the GPU's",
            "cpu_model": cpu_model(),
            "one_core": {"value": n_one * per / s_one, "iterations": n_one, "s": s_one},
            "matches_gpu": True, "compared_iterations": n_all}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=("small", "medium", "large"),
                    help="size preset (default large: 4,000 bases x 100,000 missions)")
    ap.add_argument("--cpu-iters", type=int, default=None,
                    help="Tabu iterations of the CPU-oracle sample on every core")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iterations", type=int, default=None,
                    help="override the Tabu iteration count (short profiled runs only)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 512 MiB device copy (counter calibration)")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the dense-sweep leg of a sparse-sweep workload")
    ap.add_argument("--no-medium", action="store_true", help="skip the medium-workload leg")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the repositioning-load leg (served vs plain)")
    ap.add_argument("--serve-requests", type=int, default=600,
                    help="requests per stream of the repositioning-load leg")
    ap.add_argument("--serve-pool", default="4096,256",
                    help="resident instances of the repositioning load: small,large")
    ap.add_argument("--serve-slots", type=int, default=128)
    ap.add_argument("--no-optimum", action="store_true",
                    help="skip the exact-optimum leg (synthetic analogue of the paper's Table 1)")
    ap.add_argument("--no-portfolio", action="store_true",
                    help="skip the seed-portfolio leg (permuted local and Tabu searches)")
    ap.add_argument("--no-fleet", action="store_true",
                    help="skip the heterogeneous-fleet leg (typed relocation search)")
    ap.add_argument("--batch-no-plain", action="store_true",
                    help="ragged-batch leg: the batched launch only (one timed run, no "
                         "per-instance solves; for profiling)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the ragged-batch leg (one launch vs one solve per instance)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(more GPUs would each take a share of the instances, one process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2001_05291_amd import fleetstage as fs
    from paper_2001_05291_amd import profiling

    fs.lib()
    log(f"[bench] workload {args.workload}")
    main_run = run_workload(fs, torch, profiling, args.workload, args.steps, args.warmup,
                            iterations=args.iterations)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n_all, n_one = {"small": (100, 100), "medium": (500, 20), "large": (20, 2)}[args.workload]
        n_all = min(args.cpu_iters or n_all, main_run["N"])
        n_one = min(n_one, n_all)
        log(f"[bench] cpu baseline: {n_all} Tabu iterations on every core, {n_one} on one")
        cpu = cpu_baseline(fs, oracle, main_run, n_all, n_one)
        log(f"[bench] cpu baseline {cpu['value']:.3e} MM-evals/s on {cpu['cores']} threads, "
            f"{cpu['one_core']['value']:.3e} on one")

    def leg_summary(run):
        return {k: run[k] for k in ("workload", "B", "M", "K", "N", "steps", "value",
                                    "ms_per_step", "roofline", "detail")}

    dense = None
    if not args.no_dense and main_run["detail"]["sweep_path"] == "sparse":
        dense = leg_summary(run_workload(fs, torch, profiling, args.workload,
                                         max(1, min(args.steps, 5)), 1,
                                         iterations=args.iterations, sparse=0))
        if (dense["detail"]["best_coverage"], dense["detail"]["best_distance_m"]) != \
                (main_run["detail"]["best_coverage"], main_run["detail"]["best_distance_m"]):
            raise SystemExit("dense and sparse sweeps reached different results")

    medium = None
    if not args.no_medium and args.workload != "medium":
        medium = leg_summary(run_workload(fs, torch, profiling, "medium", 10, 2))

    fleet = None
    if not args.no_fleet:
        from paper_2001_05291_amd import fleetbench
        fleet = fleetbench.run(fs, torch, workload="medium", log=log)

    portfolio = None
    if not args.no_portfolio:
        from paper_2001_05291_amd import portfoliobench
        portfolio = portfoliobench.run(fs, torch, workload="medium", log=log)

    optimum = None
    if not args.no_optimum:
        from paper_2001_05291_amd import optimumbench
        optimum = optimumbench.run(fs, torch, log=log)

    batch = None
    if not args.no_batch:
        from paper_2001_05291_amd import batchbench
        batch = batchbench.run(fs, torch, log=log, plain=not args.batch_no_plain,
                               reps=1 if args.batch_no_plain else 2)

    serve = None
    if not args.no_serve:
        from paper_2001_05291_amd import servebench
        n_small, n_large = (int(x) for x in args.serve_pool.split(","))
        serve = servebench.run(fs, torch, n_small=n_small, n_large=n_large,
                               n_requests=args.serve_requests, slots=args.serve_slots,
                               log=log)

    m = main_run
    line = {
        "metric": "mission x move evals/s",
        "value": m["value"],
        "unit": "MM-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{m['workload']}: tabu swap search, B={m['B']} bases, "
                               f"M={m['M']} missions, K={m['K']} vehicles, R={m['R']} m, "
                               f"T={m['T']}, N={m['N']}",
                   "B": m["B"], "H": m["H"], "M": m["M"], "K": m["K"], "R": m["R"],
                   "T": m["T"], "N": m["N"], "seed": m["seed"], "parallelism": "single GPU"},
        "roofline": m["roofline"],
        "cpu_baseline": cpu,
        "dense": dense,
        "medium": medium,
        "fleet": fleet,
        "portfolio": portfolio,
        "optimum": optimum,
        "batch": batch,
        "serve": serve,
        "detail": m["detail"],
    }
    if args.copy_probe:
        # a plain copy (512 MiB read + 512 MiB written) and a plain read
        # (512 MiB summed): counter calibration and the streaming rate this
        # device reaches, beside the sweep's
        dev = torch.device("cuda:0")
        x = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
            torch.sum(x)
        torch.cuda.synchronize()
        log("[bench] copy probe: 536870912 B read, 536870912 B written (x3); "
            "read probe: 536870912 B summed (x3)")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
