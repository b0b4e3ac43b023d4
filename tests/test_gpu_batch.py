"""GPU parity of the ragged batch: every instance of a batch gets exactly the
result, score and trace of its solo solve, and the oracle's."""

import numpy as np
import pytest
import torch

import oracle
from paper_2001_05291_amd import synth

from gpu_util import assert_trace_equal, oracle_table, padded_table, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    from paper_2001_05291_amd import fleetstage
    fleetstage.lib()
    return fleetstage


def same(a, b):
    assert np.array_equal(a.best_open.cpu().numpy(), b.best_open.cpu().numpy())
    assert (a.coverage, a.distance, a.best_iter) == (b.coverage, b.distance, b.best_iter)
    assert np.array_equal(a.trace, b.trace)
    assert np.array_equal(a.assign.cpu().numpy(), b.assign.cpu().numpy())


@pytest.mark.parametrize("refresh_wide,persist", [("0", "0"), ("1", "0"), ("0", "1")])
def test_batch_random_ragged_matches_solo_and_oracle(fs, monkeypatch, refresh_wide, persist):
    # per-iteration launches (both refresh widths) and the persistent search
    monkeypatch.setenv("FS_REFRESH_WIDE", refresh_wide)
    monkeypatch.setenv("FS_PERSIST", persist)
    rng = np.random.default_rng(71)
    items, hosts = [], []
    for i in range(40):
        B = int(rng.integers(1, 90))
        M = int(rng.integers(1, 800))
        K = int(rng.integers(1, min(B, 24) + 1))
        C = rng.integers(1, 5000, size=(B, M)).astype(np.int32)
        if i % 5 == 0:
            C = rng.integers(1, 6, size=(B, M)).astype(np.int32)
        R = int(rng.integers(0, 5200))
        ldc = (M + 3) // 4 * 4
        it = dict(C=padded_table(C, ldc), K=K, range_m=R, M=M)
        if i % 3 == 0:
            it["init_open"] = torch.tensor(rng.choice(B, K, replace=False), dtype=torch.int32)
        items.append(it)
        hosts.append(C)
    T, N = 6, 25
    for mode in (0, 1):
        res = fs.tabu_solve_batch(items, T, N, mode=mode)
        for it, C, r in zip(items, hosts, res):
            solo = fs.tabu_solve(it["C"], it["K"], it["range_m"], T, N, mode=mode,
                                 init_open=it.get("init_open"), M=it["M"])
            same(r, solo)
            init = None if "init_open" not in it else it["init_open"].numpy()
            o = oracle.tabu(C, it["K"], it["range_m"], T, N, mode=mode, init_open=init)
            assert np.array_equal(r.best_open.cpu().numpy(), o.best_open)
            assert_trace_equal(r.trace, o)


def test_batch_unaligned_rows_use_scalar_path(fs):
    rng = np.random.default_rng(72)
    items, hosts = [], []
    for i in range(12):
        B, M = int(rng.integers(10, 60)), int(rng.integers(50, 900))
        C = rng.integers(1, 3000, size=(B, M)).astype(np.int32)
        items.append(dict(C=padded_table(C, M + (i % 3)), K=int(rng.integers(1, 9)),
                          range_m=2500, M=M))
        hosts.append(C)
    res = fs.tabu_solve_batch(items, 4, 15)
    for it, C, r in zip(items, hosts, res):
        o = oracle.tabu(C, it["K"], it["range_m"], 4, 15)
        assert np.array_equal(r.best_open.cpu().numpy(), o.best_open)
        assert_trace_equal(r.trace, o)


def test_batch_config_sized_instances(fs):
    """The ragged 1,024-instance workload (B 30-400, M 100-5,000, K 3-24,
    R 800-1,400 km): the whole batch in one launch set, every instance
    checked against its solo solve; a sample also against the oracle."""
    sizes = synth.batch_sizes(1024)
    insts = synth.batch_instances(1024, T=10, N=200)
    dev = torch.device("cuda:0")
    items = []
    for inst, sz in zip(insts, sizes):
        C, _ = fs.build_cost_table(to_dev(inst.bases), to_dev(inst.missions))
        items.append(dict(C=C, K=sz["K"], range_m=sz["R"], M=sz["M"]))
    res = fs.tabu_solve_batch(items, 10, 200)
    rng = np.random.default_rng(5)
    check = sorted(set(rng.choice(1024, 24, replace=False).tolist()) | {0, 1023})
    for i in check:
        it = items[i]
        solo = fs.tabu_solve(it["C"], it["K"], it["range_m"], 10, 200, M=it["M"])
        same(res[i], solo)
    for i in check[:6]:
        it = items[i]
        C = it["C"][:, : it["M"]].cpu().numpy()
        o = oracle.tabu(np.ascontiguousarray(C), it["K"], it["range_m"], 10, 200)
        assert np.array_equal(res[i].best_open.cpu().numpy(), o.best_open)
        assert_trace_equal(res[i].trace, o)
    for r, sz in zip(res, sizes):
        assert 0 <= r.coverage <= sz["M"]


def test_batch_invalid_instance_named(fs):
    C = torch.ones((4, 8), dtype=torch.int32, device="cuda:0")
    with pytest.raises(fs.FleetstageError) as e:
        fs.tabu_solve_batch([dict(C=C, K=2, range_m=5), dict(C=C, K=5, range_m=5)], 1, 3)
    assert e.value.status == fs.FS_E_INVALID and "instance 1" in str(e.value)
