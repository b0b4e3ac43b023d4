"""GPU parity of the sparse sweep (sorted per-block base lists walked while
the cost is below the second-nearest open cost): the same move scores and
search trajectories as the oracle, bit for bit, forced on with FS_SPARSE=1."""

import os

import numpy as np
import pytest
import torch

import oracle
from paper_2001_05291_amd import synth

pytestmark = pytest.mark.gpu

from gpu_util import assert_trace_equal, instance_and_table, padded_table  # noqa: E402

fs = None


@pytest.fixture(scope="module", autouse=True)
def _lib():
    global fs
    from paper_2001_05291_amd import fleetstage
    fs = fleetstage
    fs.lib()
    torch.cuda.init()
    yield


class env:
    """Temporarily set launch overrides (read at every call)."""

    def __init__(self, **kv):
        self.kv = {k: str(v) for k, v in kv.items()}

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.kv}
        os.environ.update(self.kv)

    def __exit__(self, *a):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def check_scores(C, S, R, ldc=None, split=None):
    B, M = C.shape
    kv = dict(FS_SPARSE=1)
    if split is not None:
        kv["FS_SPARSE_SPLIT"] = split
    with env(**kv):
        cov, dist = fs.move_scores(padded_table(C, ldc or M), torch.tensor(S, dtype=torch.int32),
                                   R, M=M)
    ocov, odist = oracle.move_scores(C, np.array(S, dtype=np.int32), R)
    assert np.array_equal(cov.cpu().numpy(), ocov)
    assert np.array_equal(dist.cpu().numpy(), odist)


@pytest.mark.parametrize("split", [1, 3, 8])
def test_move_scores_blocks_and_chunks(split):
    inst = synth.make_instance(seed=41, B=150, H=300, M=3001)    # 3 blocks, the last partial
    C, _ = oracle.cost_table(inst.bases, inst.missions, want_cf=False)
    rng = np.random.default_rng(split)
    for K in (1, 2, 9, 40):
        S = rng.choice(150, K, replace=False).tolist()
        check_scores(C, S, 1_000_000, ldc=3004, split=split)


def test_move_scores_random_tables_with_ties():
    rng = np.random.default_rng(43)
    for trial in range(30):
        B = int(rng.integers(2, 200))
        M = int(rng.integers(1, 900))
        K = int(rng.integers(1, min(B, 64) + 1))
        if K == B:
            K = B - 1 if B > 1 else 1
        hi = 6 if trial % 3 == 0 else 5000
        C = rng.integers(1, hi, size=(B, M)).astype(np.int32)
        R = int(rng.integers(0, hi + 100))
        S = rng.choice(B, K, replace=False).tolist()
        check_scores(C, S, R, ldc=M + int(rng.integers(0, 4)), split=int(rng.integers(1, 4)))


def wide_table(rng, B, M, frac):
    """Small costs with a fraction at and above 2^26 - 2, where the list
    sort switches from 32-bit to 64-bit keys (2^26 - 2 still narrow, 2^26 - 1
    and above wide)."""
    C = rng.integers(1, 5000, size=(B, M)).astype(np.int64)
    big = rng.random((B, M)) < frac
    C[big] = rng.integers(2**26 - 2, 2**31 - 2, size=int(big.sum()))
    C[0, 0] = 2**26 - 1
    return C.astype(np.int32)


def test_move_scores_wide_costs():
    rng = np.random.default_rng(49)
    for trial in range(8):
        B = int(rng.integers(70, 200))
        M = int(rng.integers(100, 700))
        C = wide_table(rng, B, M, 0.5 if trial % 2 else 0.01)
        K = int(rng.integers(1, 40))
        R = int(rng.integers(0, 2**31 - 2))
        S = rng.choice(B, K, replace=False).tolist()
        check_scores(C, S, R, ldc=M + int(rng.integers(0, 4)), split=int(rng.integers(1, 4)))


def run_both(C, K, R, T, N, mode=0, seed=0, ldc=None, split=None):
    B, M = C.shape
    kv = dict(FS_SPARSE=1)
    if split is not None:
        kv["FS_SPARSE_SPLIT"] = split
    with env(**kv):
        g = fs.tabu_solve(padded_table(C, ldc or M), K, R, T, N, mode=mode, M=M, seed=seed)
    o = (oracle.tabu(C, K, R, T, N, mode=mode) if mode < 2
         else oracle.perm_search(C, K, R, T, N, mode, seed))
    return g, o


def assert_same(g, o, C, R):
    assert np.array_equal(g.best_open.cpu().numpy(), o.best_open)
    assert (g.coverage, g.distance, g.best_iter) == (o.coverage, o.distance, o.best_iter)
    assert_trace_equal(g.trace, o)
    assert np.array_equal(g.assign.cpu().numpy(), oracle.assign(C, o.best_open, R))


@pytest.mark.parametrize("cfg", ["small", "medium"])
def test_tabu_full_trace_configs(cfg):
    c = synth.WORKLOADS[cfg]
    _, C = instance_and_table(cfg)
    g, o = run_both(C, c["K"], c["R"], c["T"], c["N"], ldc=(c["M"] + 3) // 4 * 4)
    assert_same(g, o, C, c["R"])


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_other_modes_and_chunks(mode):
    inst = synth.make_instance(seed=44, B=200, H=400, M=5000)
    C, _ = oracle.cost_table(inst.bases, inst.missions, want_cf=False)
    for split in (1, 4):
        g, o = run_both(C, 12, 1_000_000, 5, 40, mode=mode, seed=3, split=split)
        assert_same(g, o, C, 1_000_000)


def test_random_instances():
    rng = np.random.default_rng(47)
    for trial in range(20):
        B = int(rng.integers(2, 130))
        M = int(rng.integers(1, 700))
        K = int(rng.integers(1, min(B - 1, 64) + 1)) if B > 1 else 1
        hi = 8 if trial % 4 == 0 else 5000
        C = rng.integers(1, hi, size=(B, M)).astype(np.int32)
        R = int(rng.integers(0, hi + 200))
        g, o = run_both(C, K, R, int(rng.integers(0, 9)), int(rng.integers(0, 40)),
                        ldc=M + int(rng.integers(0, 4)), split=int(rng.integers(1, 4)))
        assert_same(g, o, C, R)


def test_tabu_trace_wide_costs():
    rng = np.random.default_rng(50)
    C = wide_table(rng, 150, 900, 0.05)
    g, o = run_both(C, 9, 2**30, 5, 60, ldc=901, split=2)
    assert_same(g, o, C, 2**30)


@pytest.mark.parametrize("packed", [0, 1])
def test_packed_lists_at_the_key_boundary(packed):
    # lists packed into (cost << 6 | id) keys when every cost is below
    # 2^26 - 1, unpacked otherwise: costs just below the boundary (packed),
    # one cost on it (built again unpacked), and the second-nearest cost at
    # and beyond it (thresholds of the packed walk); also ordinary tables with
    # packing switched off
    top = 2**26 - 1
    rng = np.random.default_rng(52 + packed)
    tables = []
    C = rng.integers(top - 40, top, size=(130, 300)).astype(np.int32)
    tables.append((C, top - 20))
    C2 = C.copy()
    C2[77, 123] = top
    tables.append((C2, top))
    C3 = rng.integers(1, 60, size=(130, 300)).astype(np.int32)
    C3[:, ::7] = top - 1
    tables.append((C3, 2**31 - 2))
    tables.append((rng.integers(1, 5000, size=(97, 401)).astype(np.int32), 4000))
    for C, R in tables:
        with env(FS_SPARSE_PACKED=packed):
            g, o = run_both(C, 11, R, 4, 30, ldc=C.shape[1] + 3, split=2)
        assert_same(g, o, C, R)
        with env(FS_SPARSE_PACKED=packed):
            check_scores(C, rng.choice(C.shape[0], 11, replace=False).tolist(), R, split=3)


@pytest.mark.parametrize("fuse", [0, 1])
@pytest.mark.parametrize("mode", [0, 1, 3])
def test_fused_scoring_and_refresh(fuse, mode):
    # the block scoring and the refresh in one launch (refresh workgroups wait
    # for the scoring ones) or in two, with mission chunks and both refresh
    # widths
    inst = synth.make_instance(seed=53, B=300, H=500, M=6000)
    C, _ = oracle.cost_table(inst.bases, inst.missions, want_cf=False)
    for split, wide in ((4, 0), (3, 1)):
        with env(FS_FUSE=fuse, FS_REFRESH_SPLIT4=wide):
            g, o = run_both(C, 20, 1_000_000, 6, 50, mode=mode, seed=9, split=split)
        assert_same(g, o, C, 1_000_000)


def test_default_rule_picks_sparse_for_many_closed_bases():
    """Many closed bases and a long search take the sparse sweep by default
    (its block scoring shows up as the "finalize" timing group, or fused with
    the refresh as "score_refresh"); the result equals the dense sweep's
    record for record."""
    inst = synth.make_instance(seed=48, B=2100, H=600, M=4000)   # 3 mission chunks
    C, _ = oracle.cost_table(inst.bases, inst.missions, want_cf=False)
    Cd = padded_table(C, 4000)
    fs.timing_enable(True, every=1)
    a = fs.tabu_solve(Cd, 10, 900_000, 7, 100)
    torch.cuda.synchronize()
    _, fin = fs.timing_read("finalize")
    _, fused = fs.timing_read("score_refresh")
    fs.timing_read("sweep")
    fs.timing_read("refresh")
    fs.timing_enable(False)
    assert fin + fused > 0
    with env(FS_SPARSE=0):
        b = fs.tabu_solve(Cd, 10, 900_000, 7, 100)
    assert np.array_equal(a.best_open.cpu().numpy(), b.best_open.cpu().numpy())
    assert (a.coverage, a.distance, a.best_iter) == (b.coverage, b.distance, b.best_iter)
    assert np.array_equal(a.trace, b.trace)
    assert np.array_equal(a.assign.cpu().numpy(), b.assign.cpu().numpy())
