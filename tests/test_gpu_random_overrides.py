"""Seeded random searches under random launch geometries: every combination
of rows per workgroup, loads in flight, queued or in-place scoring,
1024-thread workgroups, mission splits, refresh width and slot split, dense or
sparse sweep, the persistent search
and the autotuner gives the oracle's trajectory bit for bit (modes 0-3,
Section 4.3; random tables, ties, costs beyond 2^26), for single instances,
ragged batches and typed fleets."""

import os

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

from gpu_util import assert_trace_equal, padded_table  # noqa: E402

fs = None

KEYS = ("FS_SWEEP_J", "FS_SWEEP_U", "FS_SWEEP_QUEUE", "FS_SWEEP_WIDE", "FS_SWEEP_SPLIT",
        "FS_REFRESH_WIDE", "FS_REFRESH_SPLIT4", "FS_SPARSE", "FS_SPARSE_SPLIT", "FS_AUTOTUNE",
        "FS_PERSIST", "FS_PERSIST_TAB", "FS_SPARSE_PACKED", "FS_FUSE")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    global fs
    from paper_2001_05291_amd import fleetstage
    fs = fleetstage
    fs.lib()
    torch.cuda.init()
    saved = {k: os.environ.get(k) for k in KEYS}
    yield
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


def draw_env(rng):
    env = {}
    if rng.random() < 0.5:
        env["FS_SWEEP_J"] = int(rng.choice([1, 2, 4, 8, 16]))
    if rng.random() < 0.5:
        env["FS_SWEEP_U"] = int(rng.choice([1, 2, 4]))
    if rng.random() < 0.5:
        env["FS_SWEEP_QUEUE"] = int(rng.integers(0, 2))
    if rng.random() < 0.3:
        env["FS_SWEEP_WIDE"] = int(rng.integers(0, 2))
    if rng.random() < 0.3:
        env["FS_SWEEP_SPLIT"] = int(rng.integers(1, 5))
    if rng.random() < 0.3:
        env["FS_REFRESH_WIDE"] = int(rng.integers(0, 2))
    if rng.random() < 0.3:
        env["FS_REFRESH_SPLIT4"] = int(rng.integers(0, 2))
    if rng.random() < 0.4:
        env["FS_SPARSE"] = int(rng.integers(0, 2))
    if rng.random() < 0.5:
        env["FS_PERSIST"] = int(rng.integers(0, 2))
    if rng.random() < 0.3:
        env["FS_PERSIST_TAB"] = int(rng.integers(0, 2))
    if rng.random() < 0.3:
        env["FS_SPARSE_SPLIT"] = int(rng.integers(1, 4))
    if rng.random() < 0.3:
        env["FS_SPARSE_PACKED"] = int(rng.integers(0, 2))
    if rng.random() < 0.3:
        env["FS_FUSE"] = int(rng.integers(0, 2))
    env["FS_AUTOTUNE"] = int(rng.integers(0, 2))
    return env


@pytest.mark.parametrize("seed", range(4))
def test_random_searches_under_random_geometries(seed):
    rng = np.random.default_rng(1000 + seed)
    for case in range(30):
        for k in KEYS:
            os.environ.pop(k, None)
        env = draw_env(rng)
        os.environ.update({k: str(v) for k, v in env.items()})
        B = int(rng.integers(2, 260))
        M = int(rng.integers(1, 1500))
        K = int(rng.integers(1, min(B, 64) + 1))
        if K == B and B > 1:
            K = B - 1
        hi = int(rng.choice([6, 5000, 2**27]))
        C = rng.integers(1, hi, size=(B, M)).astype(np.int32)
        R = int(rng.integers(0, hi + 100))
        T = int(rng.integers(0, 12))
        N = int(rng.integers(0, 80))
        mode = int(rng.integers(0, 4))
        sd = int(rng.integers(0, 2**40))
        ldc = M + int(rng.integers(0, 5))
        what = dict(case=case, env=env, B=B, M=M, K=K, hi=hi, R=R, T=T, N=N, mode=mode)
        g = fs.tabu_solve(padded_table(C, ldc), K, R, T, N, mode=mode, M=M, seed=sd)
        o = (oracle.tabu(C, K, R, T, N, mode=mode) if mode < 2
             else oracle.perm_search(C, K, R, T, N, mode, sd))
        assert np.array_equal(g.best_open.cpu().numpy(), o.best_open), what
        assert (g.coverage, g.distance, g.best_iter) == (o.coverage, o.distance, o.best_iter), what
        assert_trace_equal(g.trace, o)
        assert np.array_equal(g.assign.cpu().numpy(), oracle.assign(C, o.best_open, R)), what


def set_env(rng):
    for k in KEYS:
        os.environ.pop(k, None)
    env = draw_env(rng)
    env.pop("FS_SPARSE", None)        # (the sparse sweep takes single instances only)
    env.pop("FS_SPARSE_SPLIT", None)
    os.environ.update({k: str(v) for k, v in env.items()})
    return env


@pytest.mark.parametrize("seed", range(2))
def test_random_batches_under_random_geometries(seed):
    """Ragged batches (one launch set, modes 0-3) give each instance's
    oracle result and trajectory."""
    rng = np.random.default_rng(2000 + seed)
    for case in range(8):
        env = set_env(rng)
        mode = int(rng.integers(0, 4))
        T = int(rng.integers(0, 10))
        N = int(rng.integers(0, 40))
        items, hosts = [], []
        for i in range(int(rng.integers(1, 24))):
            B = int(rng.integers(2, 120))
            M = int(rng.integers(1, 600))
            K = int(rng.integers(1, min(B - 1, 40) + 1))
            hi = int(rng.choice([6, 5000]))
            C = rng.integers(1, hi, size=(B, M)).astype(np.int32)
            items.append(dict(C=padded_table(C, M + int(rng.integers(0, 4))), K=K,
                              range_m=int(rng.integers(0, hi + 100)), M=M,
                              seed=int(rng.integers(0, 2**40))))
            hosts.append(C)
        res = fs.tabu_solve_batch(items, T, N, mode=mode)
        for idx, (it, C, r) in enumerate(zip(items, hosts, res)):
            what = dict(case=case, instance=idx, env=env, mode=mode, T=T, N=N)
            o = (oracle.tabu(C, it["K"], it["range_m"], T, N, mode=mode) if mode < 2 else
                 oracle.perm_search(C, it["K"], it["range_m"], T, N, mode, it["seed"]))
            assert np.array_equal(r.best_open.cpu().numpy(), o.best_open), what
            assert (r.coverage, r.distance, r.best_iter) == (o.coverage, o.distance,
                                                             o.best_iter), what
            assert_trace_equal(r.trace, o)


@pytest.mark.parametrize("seed", range(2))
def test_random_fleets_under_random_geometries(seed):
    """Typed fleets (Section 3's heterogeneous model, modes 0-1) under random
    launch geometries give the typed oracle's result and trajectory."""
    rng = np.random.default_rng(3000 + seed)
    done = 0
    while done < 20:
        env = set_env(rng)
        B = int(rng.integers(3, 120))
        M = int(rng.integers(1, 800))
        hel = (rng.random(B) < 0.4).astype(np.int32)
        rho = (rng.random(M) < 0.3).astype(np.int32) if rng.random() < 0.8 else None
        aero = int((hel == 0).sum())
        K_f = int(rng.integers(0, min(aero, B - 1) + 1))
        K_r = int(rng.integers(0 if K_f else 1, min(B - K_f, 40) + 1))
        if K_r + K_f > B or aero + min(int(hel.sum()), K_r) < K_r + K_f:
            continue
        hi = int(rng.choice([8, 5000]))
        C = rng.integers(1, hi, size=(B, M)).astype(np.int32)
        R = int(rng.integers(0, hi + 200))
        T = int(rng.integers(0, 10))
        N = int(rng.integers(0, 40))
        mode = int(rng.integers(0, 2))
        what = dict(env=env, B=B, M=M, K_r=K_r, K_f=K_f, mode=mode)
        g = fs.fleet_solve(padded_table(C, M + int(rng.integers(0, 4))), K_r, K_f, hel, rho, R,
                           T, N, mode=mode, M=M)
        o = oracle.fleet_tabu(C, K_r, K_f, hel, rho if rho is not None else np.zeros(M, np.int32),
                              R, T, N, mode=mode)
        assert np.array_equal(g.best_open.cpu().numpy(), o.best_open), what
        assert np.array_equal(g.best_rotary.cpu().numpy(), o.best_rot), what
        assert (g.coverage, g.distance, g.best_iter) == (o.coverage, o.distance, o.best_iter), what
        assert_trace_equal(g.trace, o)
        done += 1
