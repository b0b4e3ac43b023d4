"""A synthetic analogue of the paper's evaluation against the exact optimum
(Section 5: Table 1 and Figs. 2-3), with the GPU enumeration standing in for
the exact solver.

Eleven datasets of 10, 20, ..., 110 missions over 40 candidate bases and 120
hospitals (the generator of the workloads, dataset d seeded with d) place 4
vehicles (the paper's 12 of 378 bases is beyond enumeration).  The range
exceeds every cost, so every mission is served and the objective is the total
distance, as in the paper's model.  Per dataset: the optimum by enumeration,
the base ranking, the average of 100 random placements (Fig. 2), and ten seeds
each of the permuted local search and permuted Tabu search as one batch launch
(Table 1: upper / lower / average gap to the optimum), beside the
deterministic Tabu search.  Gaps are (distance - optimum) / optimum in %.
"""

from __future__ import annotations

import time

import numpy as np

from . import synth

B_BASES, H_HOSP, K_VEH = 40, 120, 4
MISSIONS = tuple(range(10, 111, 10))
RANGE_ALL = 2**31 - 2     # above every cost: all missions served
T, N, SEEDS, RANDOM_STARTS = 3, 200, 10, 100


def _gap(d, opt):
    return 100.0 * (d - opt) / opt


def _ula(vals):
    a = np.asarray(vals, dtype=np.float64)
    return {"upper": float(a.max()), "lower": float(a.min()), "average": float(a.mean())}


def run(fs, torch, log=print):
    dev = torch.device("cuda:0")
    rows = []
    enum_placements = 0
    enum_s = 0.0
    for d, M in enumerate(MISSIONS):
        inst = synth.make_instance(seed=d, B=B_BASES, H=H_HOSP, M=M)
        C, _ = fs.build_cost_table(torch.from_numpy(inst.bases).to(dev),
                                   torch.from_numpy(inst.missions).to(dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        best, cov, opt, n = fs.brute_optimum(C, K_VEH, RANGE_ALL)
        torch.cuda.synchronize()
        enum_s += time.perf_counter() - t0
        enum_placements += n
        if cov != M:
            raise RuntimeError(f"dataset {d}: the optimum leaves missions unserved")
        rank = fs.tabu_solve(C, K_VEH, RANGE_ALL, T, 0, want_assign=False, want_trace=False)
        rng = np.random.default_rng(1000 + d)
        rnd = []
        for _ in range(RANDOM_STARTS):
            S = torch.from_numpy(rng.choice(B_BASES, K_VEH, replace=False).astype(np.int32))
            r = fs.tabu_solve(C, K_VEH, RANGE_ALL, T, 0, init_open=S, want_assign=False,
                              want_trace=False)
            rnd.append(r.distance)
        tabu = fs.tabu_solve(C, K_VEH, RANGE_ALL, T, N, want_assign=False, want_trace=False)
        row = {"missions": M, "optimum_m": opt, "optimum_bases": best.cpu().tolist(),
               "base_ranking_gap": _gap(rank.distance, opt),
               "random_start_gap": _gap(float(np.mean(rnd)), opt),
               "tabu_gap": _gap(tabu.distance, opt)}
        for name, mode in (("perm_local", fs.MODE_PERM_LOCAL), ("perm_tabu", fs.MODE_PERM_TABU)):
            items = [dict(C=C, K=K_VEH, range_m=RANGE_ALL, seed=s) for s in range(SEEDS)]
            res = fs.tabu_solve_batch(items, T, N, mode=mode, want_assign=False,
                                      want_trace=False)
            row[name + "_gap"] = _ula([_gap(x.distance, opt) for x in res])
        rows.append(row)
    log(f"[optimum] {len(rows)} datasets; enumeration {enum_placements} placements in "
        f"{enum_s:.3f} s; permuted Tabu average gap "
        f"{np.mean([r['perm_tabu_gap']['average'] for r in rows]):.2f}%")
    return {"bases": B_BASES, "vehicles": K_VEH, "seeds": SEEDS, "random_starts": RANDOM_STARTS,
            "enumeration_placements_per_s": enum_placements / enum_s, "datasets": rows}
