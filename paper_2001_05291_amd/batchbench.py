"""The ragged batch on one GPU: one launch set against one solve per instance.

1,024 instances of uneven size (B in [30, 400], M in [100, 5,000], K in
[3, 24], per-instance range), tenure 10 and 200 iterations each.  Tables are
built and resident before timing.  The plain path calls ``tabu_solve`` once
per instance; the batched path calls ``tabu_solve_batch`` once for all of
them.  Both results must be identical for every instance.
"""

from __future__ import annotations

import time

import numpy as np

from . import synth


def run(fs, torch, n: int | None = None, reps: int = 2, log=print, plain: bool = True):
    cfg = synth.BATCH
    n = cfg["n"] if n is None else n
    T, N = cfg["T"], cfg["N"]
    log(f"[batch] {n} instances, T={T}, N={N}")
    insts = synth.batch_instances(n, cfg["size_seed"], T, N)
    dev = torch.device("cuda:0")
    tables = []
    for w in insts:
        C, _ = fs.build_cost_table(torch.from_numpy(w.bases).to(dev),
                                   torch.from_numpy(w.missions).to(dev))
        tables.append(C)
    torch.cuda.synchronize()
    evals = sum(N * w.K * (w.B - w.K) * w.M for w in insts)
    bytes_per_iter = sum(4 * (w.B - w.K) * w.M for w in insts)

    def plain_solves():
        return [fs.tabu_solve(C, w.K, w.R, T, N, want_assign=False, want_trace=False)
                for C, w in zip(tables, insts)]

    items = [dict(C=C, K=w.K, range_m=w.R) for C, w in zip(tables, insts)]

    def batched():
        return fs.tabu_solve_batch(items, T, N, want_assign=False, want_trace=False)

    def timed(f):
        best, out = None, None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = f()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return out, best

    batched()   # warm-up
    pl, t_plain = timed(plain_solves) if plain else (None, None)
    ba, t_batch = timed(batched)
    # per-launch device time of the batched iteration's two kernels (every
    # 16th launch stamped)
    fs.timing_enable(True, every=16)
    batched()
    torch.cuda.synchronize()
    sweep_ms, sweep_n = fs.timing_read("sweep")
    refresh_ms, refresh_n = fs.timing_read("refresh")
    fs.timing_enable(False)
    bad = 0
    for a, b in zip(pl or [], ba):
        same = (np.array_equal(a.best_open.cpu().numpy(), b.best_open.cpu().numpy())
                and (a.coverage, a.distance, a.best_iter) == (b.coverage, b.distance, b.best_iter))
        bad += not same
    if plain:
        log(f"[batch] plain {n / t_plain:.1f} solves/s, batched {n / t_batch:.1f} solves/s, "
            f"{bad} mismatches")
    else:
        log(f"[batch] batched {n / t_batch:.1f} solves/s (plain path not run)")
    return {"instances": n, "T": T, "N": N,
            "plain": ({"solves_per_s": n / t_plain, "s": t_plain,
                       "mm_evals_per_s": evals / t_plain} if plain else None),
            "batched": {"solves_per_s": n / t_batch, "s": t_batch,
                        "mm_evals_per_s": evals / t_batch,
                        "sweep_bytes_per_iteration": bytes_per_iter,
                        "sweep_us_per_launch": 1e3 * sweep_ms / max(sweep_n, 1),
                        "refresh_us_per_launch": 1e3 * refresh_ms / max(refresh_n, 1),
                        "sweep_gb_per_s": bytes_per_iter / max(sweep_ms / max(sweep_n, 1), 1e-9)
                        / 1e6},
            "identical": (bad == 0) if plain else None, "mismatched_instances": bad}
