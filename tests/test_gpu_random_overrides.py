"""Seeded random searches under random launch geometries: every combination
of rows per workgroup, loads in flight, queued or in-place scoring,
1024-thread workgroups, mission splits, refresh width, dense or sparse sweep
and the autotuner gives the oracle's trajectory bit for bit (modes 0-3,
Section 4.3; random tables, ties, costs beyond 2^26)."""

import os

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

from gpu_util import assert_trace_equal, padded_table  # noqa: E402

fs = None

KEYS = ("FS_SWEEP_J", "FS_SWEEP_U", "FS_SWEEP_QUEUE", "FS_SWEEP_WIDE", "FS_SWEEP_SPLIT",
        "FS_REFRESH_WIDE", "FS_SPARSE", "FS_SPARSE_SPLIT", "FS_AUTOTUNE")


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
        env["FS_SWEEP_J"] = int(rng.choice([1, 2, 4, 8]))
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
    if rng.random() < 0.4:
        env["FS_SPARSE"] = int(rng.integers(0, 2))
    if rng.random() < 0.3:
        env["FS_SPARSE_SPLIT"] = int(rng.integers(1, 4))
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
