"""The heterogeneous fleet on one GPU: the typed relocation search on a
workload instance with heliports and rotary-only missions.

The instance is a single-instance workload (cost table built and resident
before timing) with seeded base and mission kinds (``synth.fleet_flags``) and
the fleet split into rotary- and fixed-wing vehicles by ``synth.fleet_split``;
the search starts from the typed base ranking.  Reported: solves/s and
iterations/s, the mission x move evaluations per second (every iteration
scores each vehicle against every closed base it may use), and the typed
sweep's algorithmic bytes per launch over its event-timed launch time.
"""

from __future__ import annotations

import time

import numpy as np

from . import synth

HBM_PEAK_GBS = 8000.0


def run(fs, torch, workload: str = "medium", reps: int = 3, log=print):
    c = synth.WORKLOADS[workload]
    B, M, K, R, T, N = c["B"], c["M"], c["K"], c["R"], c["T"], c["N"]
    inst = synth.workload_instance(workload)
    hel, rho = synth.fleet_flags(c["seed"], B, inst.mission_ph, c["H"])
    K_r, K_f = synth.fleet_split(K)
    log(f"[fleet] {workload}: B={B} ({int(hel.sum())} heliports) M={M} "
        f"({int(rho.sum())} rotary-only) K_r={K_r} K_f={K_f} T={T} N={N}")
    dev = torch.device("cuda:0")
    C, _ = fs.build_cost_table(torch.from_numpy(inst.bases).to(dev),
                               torch.from_numpy(inst.missions).to(dev))
    hel_d = torch.from_numpy(hel).to(dev)
    rho_d = torch.from_numpy(rho).to(dev)
    torch.cuda.synchronize()

    def solve():
        return fs.fleet_solve(C, K_r, K_f, hel_d, rho_d, R, T, N, want_assign=False,
                              want_trace=False)

    solve()   # warm-up
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        t0 = time.perf_counter()
        r = solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    fs.timing_enable(True, every=8)
    r = solve()
    torch.cuda.synchronize()
    sweep_ms, sweep_n = fs.timing_read("sweep")
    refresh_ms, refresh_n = fs.timing_read("refresh")
    fs.timing_enable(False)
    # moves per iteration: a rotary-wing vehicle to any closed base, a
    # fixed-wing one to a closed aerodrome (counted on the final placement;
    # the number of closed aerodromes changes by at most one per move)
    open_ids = r.best_open.cpu().numpy()
    closed = np.ones(B, dtype=bool)
    closed[open_ids] = False
    moves = K_r * int(closed.sum()) + K_f * int((closed & (hel == 0)).sum())
    sweep_bytes = (B - K) * M * 4 + 12 * M
    sweep_s = (sweep_ms / max(sweep_n, 1)) / 1e3
    achieved = sweep_bytes / sweep_s / 1e9 if sweep_n else None
    log(f"[fleet] {1 / best:.1f} solves/s, {N / best:.0f} iterations/s, "
        f"sweep {1e6 * sweep_s:.1f} us/launch")
    return {"workload": f"{workload} with {int(hel.sum())} heliports, "
                        f"{int(rho.sum())} rotary-only missions, K_r={K_r}, K_f={K_f}",
            "solves_per_s": 1 / best, "iterations_per_s": N / best,
            "mm_evals_per_s": N * moves * M / best,
            "coverage": r.coverage, "distance_m": r.distance, "best_iter": r.best_iter,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS if achieved else None,
                         "kernel": "k_sweep (typed)", "bytes_per_launch": sweep_bytes,
                         "avg_launch_us": 1e6 * sweep_s, "launches": sweep_n},
            "refresh_us_per_launch": 1e3 * refresh_ms / max(refresh_n, 1)}
