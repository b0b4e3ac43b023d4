#!/usr/bin/env python3
"""Throughput of the fleet-staging hot path on one MI355X.

One step = the whole hot path over one synthetic instance: the FP64 haversine
cost table, base ranking, and the Tabu search for its full iteration count.
The default workload is 500 bases, 1,500 hospitals, 20,000 missions,
30 vehicles, range 1,000 km, tenure 15, 500 iterations.

The metric is mission x move evaluations per second: every Tabu iteration
scores K*(B-K) swap moves over M missions.  It is reported for the whole step
(cost table and ranking included in the time).  Alongside:
  roofline      the swap sweep's algorithmic bytes per launch over its average
                launch time (HIP events on its own stream), against 8 TB/s HBM;
  cpu_baseline  the CPU oracle on a bounded sample of the same search;
  fleet         the heterogeneous fleet (heliports, rotary-only missions,
                rotary- and fixed-wing vehicles) on the same workload: the
                typed relocation search's solves/s and its sweep roofline;
  portfolio     the paper's permuted local and Tabu searches (random scan
                orders), ten seeds each in one batch launch: runs/s and the
                upper / lower / average result;
  optimum       a synthetic analogue of the paper's Table 1 and Fig. 2:
                eleven small datasets against their exact optimum by GPU
                enumeration (base ranking, random starts, ten-seed local and
                Tabu searches: upper / lower / average gap);
  batch         the ragged batch (1,024 instances of uneven size, 200
                iterations each): solves/s of one launch set against one solve
                per instance, results identical;
  serve         the repositioning load (95% small / 5% large instances, 10% of
                the missions redrawn, 100 warm-started iterations per request):
                solves/s at saturation and p50/p99 latency under Poisson
                arrivals at 0.5/0.8/1.0x the plain path's saturation rate, for
                the plain path (one table build + one solve per request) and
                the server, whose results must be identical.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="medium", choices=("small", "medium", "large"),
                    help="size preset (default medium: 500 bases x 20,000 missions)")
    ap.add_argument("--cpu-iters", type=int, default=None,
                    help="Tabu iterations of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iterations", type=int, default=None,
                    help="override the Tabu iteration count (short profiled runs only)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 512 MiB device copy (counter calibration)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the repositioning-load leg (served vs plain)")
    ap.add_argument("--serve-requests", type=int, default=600,
                    help="requests per stream of the repositioning-load leg")
    ap.add_argument("--serve-pool", default="1024,64",
                    help="resident instances of the repositioning load: small,large")
    ap.add_argument("--serve-slots", type=int, default=128)
    ap.add_argument("--no-optimum", action="store_true",
                    help="skip the exact-optimum leg (synthetic analogue of the paper's Table 1)")
    ap.add_argument("--no-portfolio", action="store_true",
                    help="skip the seed-portfolio leg (permuted local and Tabu searches)")
    ap.add_argument("--no-fleet", action="store_true",
                    help="skip the heterogeneous-fleet leg (typed relocation search)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the ragged-batch leg (one launch set vs one solve per instance)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(more GPUs would each take a share of the instances, one process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2001_05291_amd import fleetstage as fs
    from paper_2001_05291_amd import synth

    from paper_2001_05291_amd import profiling

    c = synth.WORKLOADS[args.workload]
    B, M, K, R, T, N = c["B"], c["M"], c["K"], c["R"], c["T"], c["N"]
    if args.iterations is not None:
        N = args.iterations
    log(f"[bench] building instance B={B} H={c['H']} M={M} K={K} R={R} T={T} N={N}")
    inst = synth.workload_instance(args.workload)
    dev = torch.device("cuda:0")
    bases = torch.from_numpy(inst.bases).to(dev)
    hospitals = torch.from_numpy(inst.hospitals).to(dev)
    mission_ph = torch.from_numpy(inst.mission_ph).to(dev)
    fs.lib()

    result = {}

    def step():
        # the indexed builder: missions as hospital-id pairs (the same table,
        # bitwise, as from the missions' coordinates)
        C, _ = fs.build_cost_table_indexed(bases, hospitals, mission_ph)
        r = fs.tabu_solve(C, K, R, T, N, want_assign=True, want_trace=False)
        result["r"] = r
        result["C"] = C
        return C

    for w in range(args.warmup):
        step()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    # every 8th sweep / refresh launch carries dispatch-stamped events (a
    # dispatch with events is followed by a gap, so timing all of them would
    # slow the timed loop itself)
    fs.timing_enable(True, every=8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sweep_ms, sweep_n = fs.timing_read("sweep")
    refresh_ms, refresh_n = fs.timing_read("refresh")
    fin_ms, fin_n = fs.timing_read("finalize")
    fs.timing_enable(False)
    log(f"[bench] timed {args.steps} steps in {elapsed:.4f} s")

    evals_per_step = N * K * (B - K) * M
    value = evals_per_step * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    # dominant kernel: the swap sweep.  Dense: every closed row once (4 B per
    # element) + the per-mission state (b1, b2, o1).  Sparse (its block scoring
    # runs as a second kernel, timed as "finalize"): the sorted-list entries
    # the walk needs at the final placement + the state once per base block.
    sparse = fin_n > 0
    if sparse:
        sweep_bytes = profiling.sparse_sweep_bytes(result["C"].cpu().numpy(),
                                                   result["r"].best_open.cpu().numpy())
    else:
        sweep_bytes = (B - K) * M * 4 + 12 * M
    sweep_avg_s = (sweep_ms / max(sweep_n, 1)) / 1e3
    achieved = sweep_bytes / sweep_avg_s / 1e9 if sweep_n else None
    kname = "k_sweep_sparse" if sparse else "k_sweep"
    traffic = profiling.read_traffic(
        os.path.join(ROOT, "profiles", f"{kname}_{args.workload}_traffic.md"), args.workload)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                "kernel": kname,
                "bytes_per_launch": sweep_bytes,
                "avg_launch_us": sweep_avg_s * 1e6, "launches": sweep_n}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n_cpu = args.cpu_iters or {"small": 100, "medium": 500, "large": 20}[args.workload]
        log(f"[bench] cpu baseline: oracle table + {n_cpu} Tabu iterations")
        Co, _ = oracle.cost_table(inst.bases, inst.missions, want_cf=False)
        t1 = time.perf_counter()
        oracle.tabu(Co, K, R, T, n_cpu)
        cpu_s = time.perf_counter() - t1
        cpu = {"value": n_cpu * K * (B - K) * M / cpu_s, "unit": "MM-evals/s",
               "cores": oracle.get_threads(), "kind": "oracle",
               "sample": f"first {n_cpu} of {N} Tabu iterations of the same instance "
                         f"(oracle cost table, not timed); {cpu_s:.2f} s"}
        log(f"[bench] cpu baseline {cpu['value']:.3e} MM-evals/s on {cpu['cores']} threads")

    fleet = None
    if not args.no_fleet:
        from paper_2001_05291_amd import fleetbench
        fleet = fleetbench.run(fs, torch, workload=args.workload, log=log)

    portfolio = None
    if not args.no_portfolio:
        from paper_2001_05291_amd import portfoliobench
        portfolio = portfoliobench.run(fs, torch, workload=args.workload, log=log)

    optimum = None
    if not args.no_optimum:
        from paper_2001_05291_amd import optimumbench
        optimum = optimumbench.run(fs, torch, log=log)

    batch = None
    if not args.no_batch:
        from paper_2001_05291_amd import batchbench
        batch = batchbench.run(fs, torch, log=log)

    serve = None
    if not args.no_serve:
        from paper_2001_05291_amd import servebench
        n_small, n_large = (int(x) for x in args.serve_pool.split(","))
        serve = servebench.run(fs, torch, n_small=n_small, n_large=n_large,
                               n_requests=args.serve_requests, slots=args.serve_slots,
                               log=log)

    r = result["r"]
    line = {
        "metric": "mission x move evals/s",
        "value": value,
        "unit": "MM-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: tabu swap search, B={B} bases, "
                               f"M={M} missions, K={K} vehicles, R={R} m, T={T}, N={N}",
                   "B": B, "H": c["H"], "M": M, "K": K, "R": R, "T": T, "N": N,
                   "seed": c["seed"], "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fleet": fleet,
        "portfolio": portfolio,
        "optimum": optimum,
        "batch": batch,
        "serve": serve,
        "detail": {"sweep_path": "sparse" if sparse else "dense",
                   "sparse_score_ms_per_launch": fin_ms / max(fin_n, 1) if sparse else None,
                   "sweep_ms_per_launch": sweep_ms / max(sweep_n, 1),
                   "refresh_ms_per_launch": refresh_ms / max(refresh_n, 1),
                   "best_coverage": r.coverage, "best_distance_m": r.distance,
                   "best_iter": r.best_iter},
    }
    if args.copy_probe:
        # a plain copy (512 MiB read + 512 MiB written) and a plain read
        # (512 MiB summed): counter calibration and the streaming rate this
        # device reaches, beside the sweep's
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
