"""Repositioning load on one GPU: the plain path against the server.

A request names a resident instance, redraws a tenth of its missions and runs
a warm-started Tabu search from the instance's last best placement.  The same
request streams are played through

  plain   one cost-table build and one ``tabu_solve`` per request, in arrival
          order on the calling thread (the one-solve-per-launch path);
  served  ``Server``: tables stay resident, only the redrawn columns are
          recomputed, and requests that arrive while others run join the next
          batched iteration.

Each stream is played at saturation (every request at time 0) and as Poisson
arrivals at fractions of the plain path's saturation rate; the saturation
stream is played once more on a server whose HBM budget (1 GiB) forces it to
evict and rebuild tables.  Latency runs from
a request's arrival to its result.  Every served result is compared with the
plain result of the same request, which must be identical.
"""

from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import synth


@dataclass
class Request:
    inst: int
    ids: np.ndarray      # redrawn mission ids (ascending)
    pd: np.ndarray       # their new pickup/delivery coordinates (n x 4)


def make_requests(pool, targets, seed: int, fraction: float, first: int):
    out = []
    for q, i in enumerate(targets):
        w = pool[int(i)]
        ids, pairs = synth.perturbation(seed, w.hospitals.shape[0], w.M, fraction,
                                        request=first + q)
        out.append(Request(int(i), ids, synth.missions_from_pairs(w.hospitals, pairs)))
    return out


def _wait_until(t):
    while True:
        dt = t - time.perf_counter()
        if dt <= 0:
            return
        if dt > 5e-4:
            time.sleep(dt - 3e-4)


def _summary(lat_s, elapsed_s):
    lat = np.asarray(lat_s) * 1e3
    return {"solves_per_s": len(lat) / elapsed_s, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "elapsed_s": elapsed_s}


class PlainPath:
    """One cost-table build and one tabu_solve per request."""

    def __init__(self, fs, torch, pool, T, N):
        self.fs, self.torch, self.pool, self.T, self.N = fs, torch, pool, T, N
        self.dev = torch.device("cuda:0")
        self.coords = [w.missions.copy() for w in pool]
        self.bases = [torch.from_numpy(w.bases).to(self.dev) for w in pool]
        self.prev = []
        # warm start of each instance's first request: the base ranking of its
        # initial table (what a zero-iteration solve returns)
        for i, w in enumerate(pool):
            C, _ = fs.build_cost_table(self.bases[i], torch.from_numpy(self.coords[i]).to(self.dev))
            self.prev.append(fs.rank_bases(C, w.K)[0])
        torch.cuda.synchronize()

    def solve(self, r: Request):
        fs, torch = self.fs, self.torch
        w = self.pool[r.inst]
        c = self.coords[r.inst]
        c[r.ids] = r.pd
        C, _ = fs.build_cost_table(self.bases[r.inst], torch.from_numpy(c).to(self.dev))
        res = fs.tabu_solve(C, w.K, w.R, self.T, self.N, init_open=self.prev[r.inst],
                            want_trace=False, want_assign=False)
        self.prev[r.inst] = res.best_open
        return (res.best_open.cpu().numpy(), res.coverage, res.distance, res.best_iter)

    def play(self, reqs, arrivals):
        out, lat = [], []
        t0 = time.perf_counter()
        for r, a in zip(reqs, arrivals):
            _wait_until(t0 + a)
            out.append(self.solve(r))
            lat.append(time.perf_counter() - (t0 + a))
        return out, _summary(lat, time.perf_counter() - t0)


class ServedPath:
    """The repositioning server over the same pool."""

    def __init__(self, fs, pool, T, N, slots, budget):
        self.sv = fs.Server(hbm_budget_bytes=budget, max_slots=slots)
        self.T, self.N = T, N
        self.iid = [self.sv.register(w.bases, w.missions, w.K, w.R) for w in pool]
        empty_ids = np.zeros(0, dtype=np.int32)
        empty_pd = np.zeros((0, 4))
        warm = [self.sv.submit(i, empty_ids, empty_pd, T, 0) for i in self.iid]
        for t in warm:
            self.sv.wait(t, timeout=600.0)

    def play(self, reqs, arrivals):
        sv = self.sv
        tickets, lag = [], []
        t0 = time.perf_counter()
        for r, a in zip(reqs, arrivals):
            _wait_until(t0 + a)
            lag.append(time.perf_counter() - (t0 + a))
            tickets.append(sv.submit(self.iid[r.inst], r.ids, r.pd, self.T, self.N))
        res = [sv.wait(t, timeout=600.0) for t in tickets]
        lat = [g + x.latency_s for g, x in zip(lag, res)]
        end = max(a + l for a, l in zip(arrivals, lat))
        out = [(x.best_open, x.coverage, x.distance, x.best_iter) for x in res]
        return out, _summary(lat, float(end))

    def close(self):
        stats = self.sv.stats()
        self.sv.close()
        return stats


def _mismatches(a, b):
    bad = 0
    for x, y in zip(a, b):
        if not (np.array_equal(x[0], y[0]) and tuple(x[1:]) == tuple(y[1:])):
            bad += 1
    return bad


def run(fs, torch, n_small=4096, n_large=256, n_requests=600, fractions=(0.5, 0.8, 1.0),
        slots=128, budget=200 << 30, evict_budget=1 << 30, log=print):
    cfg = synth.SERVE
    T, N, seed = cfg["T"], cfg["N"], cfg["seed"]
    log(f"[serve] pool: {n_small} small + {n_large} large instances")
    pool = synth.serve_pool(n_small, n_large)
    resident = sum(w.B * w.M * 4 for w in pool)

    # request streams: saturation first, then Poisson at fractions of the
    # plain path's saturation rate (known once the first stream has played)
    legs = [("saturation", 0.0)] + [(f"{f:g}x", f) for f in fractions]
    streams = []
    for k in range(len(legs)):
        _, targets = synth.request_stream(n_requests, 0.0, n_small, n_large, seed=seed + k,
                                          large_fraction=cfg["large_fraction"])
        streams.append(make_requests(pool, targets, seed, cfg["redraw_fraction"],
                                     first=k * n_requests))

    log("[serve] plain path: warm start lists")
    plain = PlainPath(fs, torch, pool, T, N)
    plain_res, plain_sum, arrivals = [], {}, []
    sat_rate = None
    for k, (name, f) in enumerate(legs):
        if f == 0.0:
            arr = np.zeros(n_requests)
        else:
            arr, _ = synth.request_stream(n_requests, f * sat_rate, n_small, n_large,
                                          seed=seed + k, large_fraction=cfg["large_fraction"])
        arrivals.append(arr)
        out, sm = plain.play(streams[k], arr)
        if f == 0.0:
            sat_rate = sm["solves_per_s"]
        else:
            sm["rate_per_s"] = f * sat_rate
        plain_res.append(out)
        plain_sum[name] = sm
        log(f"[serve] plain {name}: {sm['solves_per_s']:.1f} solves/s, "
            f"p50 {sm['p50_ms']:.2f} ms, p99 {sm['p99_ms']:.2f} ms")
    del plain
    torch.cuda.synchronize()

    log("[serve] server: registering and warming the pool")
    served = ServedPath(fs, pool, T, N, slots, budget)
    served_sum, bad = {}, 0
    try:
        for k, (name, f) in enumerate(legs):
            out, sm = served.play(streams[k], arrivals[k])
            if f:
                sm["rate_per_s"] = f * sat_rate
            served_sum[name] = sm
            bad += _mismatches(out, plain_res[k])
            log(f"[serve] served {name}: {sm['solves_per_s']:.1f} solves/s, "
                f"p50 {sm['p50_ms']:.2f} ms, p99 {sm['p99_ms']:.2f} ms")
    finally:
        stats = served.close()

    # the saturation stream again on a fresh server under a 1 GB budget: about
    # two large tables fit, so admissions evict idle tables (least recently
    # used first) and rebuild them on their next request
    evict = None
    if evict_budget:
        log(f"[serve] server under a {evict_budget / 2 ** 30:g} GiB budget: warming the pool")
        small = ServedPath(fs, pool, T, N, slots, evict_budget)
        try:
            out, sm = small.play(streams[0], arrivals[0])
        finally:
            est = small.close()
        ebad = _mismatches(out, plain_res[0])
        evict = {"budget_gb": evict_budget / 2 ** 30, "stream": legs[0][0], **sm,
                 "identical": ebad == 0, "mismatched_requests": ebad,
                 "server_stats": {k: est[k] for k in ("evictions", "rebuilds", "steps",
                                                      "completed")}}
        log(f"[serve] served {legs[0][0]} under the small budget: {sm['solves_per_s']:.1f} "
            f"solves/s, {est['evictions']} evictions, {ebad} mismatches")
        bad += ebad
    return {
        "pool": {"small": n_small, "large": n_large, "table_gb": resident / 1e9},
        "requests_per_stream": n_requests, "T": T, "N": N, "slots": slots,
        "budget_gb": budget / 2 ** 30, "large_fraction": cfg["large_fraction"],
        "redraw_fraction": cfg["redraw_fraction"],
        "plain": plain_sum, "served": served_sum,
        "identical": bad == 0, "mismatched_requests": bad,
        "server_stats": {k: stats[k] for k in ("evictions", "rebuilds", "steps", "completed")},
        "eviction": evict,
    }
