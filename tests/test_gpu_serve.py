"""GPU tests of the repositioning server: every request's result equals the
plain path (one tabu_solve per request, replayed in order with the same
redraws and warm starts), whatever the number of slots and with evictions;
and chains of warm-started requests against the CPU oracle."""

import numpy as np
import pytest
import torch

import oracle
from paper_2001_05291_amd import synth

from gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    from paper_2001_05291_amd import fleetstage
    fleetstage.lib()
    return fleetstage


def make_workload(n_inst, n_req, seed, sizes=((20, 120), (100, 1500), (2, 12))):
    rng = np.random.default_rng(seed)
    insts = []
    for i in range(n_inst):
        B = int(rng.integers(*sizes[0]))
        M = int(rng.integers(*sizes[1]))
        K = int(rng.integers(sizes[2][0], min(sizes[2][1], B - 1) + 1))
        R = int(rng.integers(800_000, 1_400_000))
        inst = synth.make_instance(seed=100 + i, B=B, H=3 * B, M=M)
        insts.append(dict(inst=inst, K=K, R=R))
    reqs = []
    for q in range(n_req):
        i = int(rng.integers(0, n_inst))
        inst = insts[i]["inst"]
        ids, pairs = synth.perturbation(seed + i, inst.hospitals.shape[0], inst.M, 0.1, request=q)
        pd = synth.missions_from_pairs(inst.hospitals, pairs)
        reqs.append(dict(inst=i, ids=ids, pd=pd))
    return insts, reqs


def plain_replay(fs, insts, reqs, T, N, mode=0):
    """One fs.tabu_solve per request, in submission order per instance."""
    coords = [w["inst"].missions.copy() for w in insts]
    prev = [None] * len(insts)
    out = []
    for r in reqs:
        i = r["inst"]
        coords[i][r["ids"]] = r["pd"]
        w = insts[i]
        C, _ = fs.build_cost_table(to_dev(w["inst"].bases), to_dev(coords[i]))
        res = fs.tabu_solve(C, w["K"], w["R"], T, N, mode=mode, init_open=prev[i],
                            M=w["inst"].M, want_trace=False, want_assign=False)
        prev[i] = res.best_open.clone()
        out.append((res.best_open.cpu().numpy(), res.coverage, res.distance, res.best_iter))
    return out


def serve_all(fs, insts, reqs, T, N, mode=0, **cfg):
    with fs.Server(**cfg) as sv:
        ids = [sv.register(w["inst"].bases, w["inst"].missions, w["K"], w["R"]) for w in insts]
        tickets = [sv.submit(ids[r["inst"]], r["ids"], r["pd"], T, N, mode) for r in reqs]
        res = [sv.wait(t) for t in tickets]
        stats = sv.stats()
    return res, stats


def assert_same(served, plain):
    for k, (s, p) in enumerate(zip(served, plain)):
        assert np.array_equal(s.best_open, p[0]), k
        assert (s.coverage, s.distance, s.best_iter) == p[1:], k


@pytest.mark.parametrize("slots", [1, 4, 64])
def test_served_equals_plain(fs, slots):
    insts, reqs = make_workload(6, 24, seed=1)
    plain = plain_replay(fs, insts, reqs, T=5, N=30)
    served, stats = serve_all(fs, insts, reqs, T=5, N=30, max_slots=slots)
    assert_same(served, plain)
    assert stats["completed"] == 24 and stats["running"] == 0 and stats["queued"] == 0
    assert all(s.latency_s > 0 for s in served)


def test_two_sweep_classes_in_one_round(fs, monkeypatch):
    """Instances with at least 16 closed bases and short rows are swept four
    rows per workgroup, the others one row per workgroup, as two tile classes
    in the same rounds; then again with the many-rows threshold lowered so the
    rule's other branch is taken too, each with in-place and queued scoring,
    and with long-row instances as a third class."""
    insts, reqs = make_workload(8, 32, seed=7, sizes=((8, 60), (100, 1500), (2, 12)))
    ncl = [w["inst"].B - w["K"] for w in insts]
    assert any(n >= 16 for n in ncl) and any(n < 16 for n in ncl)
    plain = plain_replay(fs, insts, reqs, T=5, N=30)
    served, _ = serve_all(fs, insts, reqs, T=5, N=30, max_slots=4)
    assert_same(served, plain)
    monkeypatch.setenv("FS_SERVE_TALL_ROWS", "10")
    served, _ = serve_all(fs, insts, reqs, T=5, N=30, max_slots=4)
    assert_same(served, plain)
    # and both with queued scoring (the default scores in place)
    monkeypatch.setenv("FS_SERVE_QUEUE", "1")
    served, _ = serve_all(fs, insts, reqs, T=5, N=30, max_slots=4)
    assert_same(served, plain)
    monkeypatch.delenv("FS_SERVE_TALL_ROWS")
    served, _ = serve_all(fs, insts, reqs, T=5, N=30, max_slots=4)
    assert_same(served, plain)
    # four-row instances with rows of at least 1,000 missions as a third
    # class (1024-thread workgroups), in place and queued
    monkeypatch.setenv("FS_SERVE_LONG_ROWS", "1000")
    served, _ = serve_all(fs, insts, reqs, T=5, N=30, max_slots=4)
    assert_same(served, plain)
    monkeypatch.setenv("FS_SERVE_QUEUE", "0")
    served, _ = serve_all(fs, insts, reqs, T=5, N=30, max_slots=4)
    assert_same(served, plain)


def test_local_search_requests(fs):
    insts, reqs = make_workload(3, 9, seed=2)
    plain = plain_replay(fs, insts, reqs, T=5, N=25, mode=1)
    served, _ = serve_all(fs, insts, reqs, T=5, N=25, mode=1, max_slots=3)
    assert_same(served, plain)


def test_eviction_keeps_results(fs):
    insts, reqs = make_workload(5, 20, seed=3, sizes=((60, 120), (1000, 2000), (3, 10)))
    plain = plain_replay(fs, insts, reqs, T=4, N=20)
    # room for about two tables and their workspaces at a time
    biggest = max(w["inst"].B * ((w["inst"].M + 3) // 4 * 4) * 4 for w in insts)
    served, stats = serve_all(fs, insts, reqs, T=4, N=20, max_slots=4,
                              hbm_budget_bytes=int(2.2 * biggest) + (512 << 10))
    assert_same(served, plain)
    assert stats["evictions"] > 0 and stats["rebuilds"] > len(insts)


def test_zero_iteration_request_and_no_redraw(fs):
    insts, reqs = make_workload(2, 4, seed=4)
    reqs[1]["ids"] = np.zeros(0, dtype=np.int32)
    reqs[1]["pd"] = np.zeros((0, 4))
    plain = plain_replay(fs, insts, reqs, T=3, N=0)
    served, _ = serve_all(fs, insts, reqs, T=3, N=0, max_slots=2)
    assert_same(served, plain)


def explain_mismatches(Cg, Co, Cfo):
    """Each int32 entry where the GPU table differs from the oracle's is one
    metre apart with the FP64 sum on a .5 rounding boundary (both roundings
    are correct there)."""
    for b, m in zip(*np.nonzero(Cg != Co)):
        assert abs(int(Cg[b, m]) - int(Co[b, m])) == 1
        assert abs(Cfo[b, m] - np.floor(Cfo[b, m]) - 0.5) <= 1e-12 * Cfo[b, m] + 1e-9


def oracle_chain(fs, w, reqs, T, N):
    """The requests of one instance replayed through the oracle in order:
    redrawn mission coordinates, the cost table, and the oracle's Tabu
    search warm-started from the previous request's best placement (the
    base ranking for the first).  The search runs on the GPU-built table,
    the shared input of the server and the oracle, after checking it against
    the oracle's own table."""
    inst = w["inst"]
    coords = inst.missions.copy()
    prev = None
    out = []
    for r in reqs:
        coords[r["ids"]] = r["pd"]
        Cg, Cfg = fs.build_cost_table(to_dev(inst.bases), to_dev(coords), want_cf=True)
        Cg = Cg.cpu().numpy()
        Cfg = Cfg.cpu().numpy()
        Co, Cfo = oracle.cost_table(inst.bases, coords)
        assert (np.abs(Cfg - Cfo) / Cfo).max() <= 1e-12
        explain_mismatches(Cg, Co, Cfo)
        o = oracle.tabu(Cg, w["K"], w["R"], T, N, init_open=prev)
        prev = o.best_open
        out.append(o)
    return out


def chain_workload(inst, K, R, n_req, seed):
    w = dict(inst=inst, K=K, R=R)
    reqs = []
    for q in range(n_req):
        ids, pairs = synth.perturbation(seed, inst.hospitals.shape[0], inst.M, 0.1, request=q)
        reqs.append(dict(inst=0, ids=ids, pd=synth.missions_from_pairs(inst.hospitals, pairs)))
    return w, reqs


def assert_chain(served, chain):
    for k, (s, o) in enumerate(zip(served, chain)):
        assert np.array_equal(s.best_open, o.best_open), k
        assert (s.coverage, s.distance, s.best_iter) == (o.coverage, o.distance, o.best_iter), k


def test_warm_start_chain_against_oracle(fs):
    """Five consecutive requests on one instance (each redraws 10% of the
    missions and warm-starts from the previous best) equal the oracle's
    chain, one request at a time and mixed with another instance's."""
    inst = synth.make_instance(seed=55, B=150, H=450, M=2400)
    w, reqs = chain_workload(inst, 11, 1_100_000, 5, seed=77)
    chain = oracle_chain(fs, w, reqs, T=10, N=100)
    served, _ = serve_all(fs, [w], reqs, T=10, N=100, max_slots=1)
    assert_chain(served, chain)
    # the same chain interleaved with requests on a second instance
    other = synth.make_instance(seed=56, B=90, H=270, M=3100)
    w2, reqs2 = chain_workload(other, 7, 1_000_000, 5, seed=78)
    for r in reqs2:
        r["inst"] = 1
    mixed = [x for pair in zip(reqs, reqs2) for x in pair]
    served, _ = serve_all(fs, [w, w2], mixed, T=10, N=100, max_slots=4)
    assert_chain(served[0::2], chain)
    assert_chain(served[1::2], oracle_chain(fs, w2, reqs2, T=10, N=100))


@pytest.mark.timeout(900)
def test_large_request_chain_against_oracle(fs):
    """Two consecutive requests on a large resident instance (2,000 bases,
    6,000 hospitals, 50,000 missions, 48 vehicles, 100 iterations, tenure
    10) equal the oracle's warm-started chain."""
    s = synth.SERVE_LARGE
    inst = synth.make_instance(seed=100_000, B=s["B"], H=s["H"], M=s["M"])
    w, reqs = chain_workload(inst, s["K"], 1_050_000, 2, seed=79)
    chain = oracle_chain(fs, w, reqs, T=synth.SERVE["T"], N=synth.SERVE["N"])
    served, _ = serve_all(fs, [w], reqs, T=synth.SERVE["T"], N=synth.SERVE["N"], max_slots=4)
    assert_chain(served, chain)


def test_failed_request_does_not_seed_warm_start(fs, monkeypatch):
    """A request reported as inconsistent (the device-side check, injected
    from the host here for the second request retired) fails with
    FS_E_INTERNAL; its redraw stays applied, but the next request on the
    instance warm-starts from the last consistent placement."""
    monkeypatch.setenv("FS_SERVE_FAIL_NTH", "2")
    insts, reqs = make_workload(1, 3, seed=11)
    w = insts[0]
    with fs.Server(max_slots=1) as sv:
        iid = sv.register(w["inst"].bases, w["inst"].missions, w["K"], w["R"])
        tickets = [sv.submit(iid, r["ids"], r["pd"], 5, 30) for r in reqs]
        first = sv.wait(tickets[0])
        with pytest.raises(fs.FleetstageError) as e:
            sv.wait(tickets[1])
        assert e.value.status == fs.FS_E_INTERNAL
        third = sv.wait(tickets[2])
    coords = w["inst"].missions.copy()
    for r in reqs:
        coords[r["ids"]] = r["pd"]
    C, _ = fs.build_cost_table(to_dev(w["inst"].bases), to_dev(coords))
    plain = fs.tabu_solve(C, w["K"], w["R"], 5, 30, init_open=torch.from_numpy(first.best_open),
                          M=w["inst"].M, want_trace=False, want_assign=False)
    assert np.array_equal(third.best_open, plain.best_open.cpu().numpy())
    assert (third.coverage, third.distance, third.best_iter) == (
        plain.coverage, plain.distance, plain.best_iter)


def test_server_errors(fs):
    inst = synth.make_instance(seed=9, B=20, H=60, M=100)
    with fs.Server(hbm_budget_bytes=1 << 30, max_slots=2) as sv:
        with pytest.raises(fs.FleetstageError) as e:
            sv.register(inst.bases, inst.missions, 21, 1_000_000)
        assert e.value.status == fs.FS_E_INVALID
        iid = sv.register(inst.bases, inst.missions, 4, 1_000_000)
        with pytest.raises(fs.FleetstageError) as e:
            sv.submit(iid + 7, [], np.zeros((0, 4)), 3, 5)
        assert e.value.status == fs.FS_E_NOTFOUND
        with pytest.raises(fs.FleetstageError) as e:
            sv.submit(iid, [100], np.zeros((1, 4)), 3, 5)
        assert e.value.status == fs.FS_E_INVALID
        with pytest.raises(fs.FleetstageError) as e:
            sv.poll((12345, iid))
        assert e.value.status == fs.FS_E_NOTFOUND
    big = synth.make_instance(seed=10, B=200, H=400, M=4000)
    with fs.Server(hbm_budget_bytes=1 << 20, max_slots=2) as sv:
        with pytest.raises(fs.FleetstageError) as e:
            sv.register(big.bases, big.missions, 5, 1_000_000)
        assert e.value.status == fs.FS_E_BUDGET
