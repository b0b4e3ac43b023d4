"""The paper's stochastic searches as a portfolio of seeds on one GPU.

Section 5 runs every search ten times with fresh random scan orders and
reports the upper, lower and average result.  Here the ten runs of the
permuted local search (mode 2) and of the permuted Tabu search (mode 3) on a
workload instance are one batch launch each (the cost table built and
resident before timing; the batch runs the iteration cap, runs that have
stopped skip their remaining iterations).  Reported per search: runs/s, the
upper / lower / average covered-mission count and total distance, the
iterations the runs took, and the deterministic Tabu search (mode 0) of the
same instance for reference.
"""

from __future__ import annotations

import time

import numpy as np

from . import synth


def _stats(vals):
    a = np.asarray(vals, dtype=np.float64)
    return {"upper": float(a.max()), "lower": float(a.min()), "average": float(a.mean())}


def run(fs, torch, workload: str = "medium", seeds: int = 10, log=print):
    c = synth.WORKLOADS[workload]
    B, M, K, R, T, N = c["B"], c["M"], c["K"], c["R"], c["T"], c["N"]
    inst = synth.workload_instance(workload)
    dev = torch.device("cuda:0")
    C, _ = fs.build_cost_table(torch.from_numpy(inst.bases).to(dev),
                               torch.from_numpy(inst.missions).to(dev))
    torch.cuda.synchronize()
    out = {"workload": workload, "seeds": seeds, "iteration_cap": N}
    ref = fs.tabu_solve(C, K, R, T, N, want_assign=False, want_trace=False)
    out["tabu"] = {"coverage": ref.coverage, "distance_m": ref.distance,
                   "best_iter": ref.best_iter}
    for name, mode in (("perm_local", fs.MODE_PERM_LOCAL), ("perm_tabu", fs.MODE_PERM_TABU)):
        items = [dict(C=C, K=K, range_m=R, seed=s) for s in range(seeds)]
        fs.tabu_solve_batch(items, T, N, mode=mode, want_assign=False, want_trace=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fs.tabu_solve_batch(items, T, N, mode=mode, want_assign=False, want_trace=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        moves = [int(r.trace["moved"].sum()) for r in res]
        stopped_at = [int(r.best_iter) for r in res]
        out[name] = {"runs_per_s": seeds / dt, "s": dt,
                     "coverage": _stats([r.coverage for r in res]),
                     "distance_m": _stats([r.distance for r in res]),
                     "moves": _stats(moves), "last_move_iter": _stats(stopped_at),
                     "distinct_results": len({(r.coverage, r.distance) for r in res})}
        log(f"[portfolio] {name}: {seeds} runs in {dt:.3f} s; coverage "
            f"{out[name]['coverage']['lower']:.0f}..{out[name]['coverage']['upper']:.0f}, "
            f"moves {out[name]['moves']['average']:.1f} on average")
    return out
