"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Integer outputs must match bit for bit; the FP64 cost
table within 1e-12 relative before rounding."""

import os

import numpy as np
import pytest
import torch

import oracle
from paper_2001_05291_amd import synth

pytestmark = pytest.mark.gpu

from gpu_util import DEV, assert_trace_equal, instance_and_table, oracle_table, padded_table, to_dev  # noqa: E402

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
    """Temporarily set launch-geometry overrides (read at every call)."""

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


# ------------------------------------------------------------------ cost table (A0)


def check_cost_table(inst, legs=3, ldc=None):
    Cg, Cfg = fs.build_cost_table(to_dev(inst.bases), to_dev(inst.missions), legs=legs,
                                  ldc=ldc, want_cf=True)
    M = inst.M
    Cg = Cg[:, :M].cpu().numpy()
    Cfg = Cfg[:, :M].cpu().numpy()
    Co, Cfo = oracle.cost_table(inst.bases, inst.missions, legs=legs)
    rel = np.abs(Cfg - Cfo) / np.maximum(Cfo, 1.0)
    assert rel.max() <= 1e-12, rel.max()
    # an int32 difference is only allowed where both FP64 values straddle a
    # rounding boundary within the tolerance
    return explain_mismatches(Cg, Co, Cfo, Cfg)


def test_cost_table_small_workload():
    assert check_cost_table(synth.workload_instance("small")) == 0


def test_cost_table_ragged_and_two_legs():
    inst = synth.make_instance(seed=21, B=37, H=90, M=1003)
    check_cost_table(inst, legs=3)
    check_cost_table(inst, legs=2, ldc=1009)


def explain_mismatches(Cg, Co, Cfo, Cfg=None):
    """Every int32 difference between two tables must be one metre where the
    FP64 sum lies within the FP64 tolerance of a .5 rounding boundary (there
    both roundings are correct).  Returns the number of such entries."""
    mism = np.nonzero(Cg != Co)
    for b, m in zip(*mism):
        assert abs(int(Cg[b, m]) - int(Co[b, m])) == 1, (b, m, Cg[b, m], Co[b, m])
        frac = Cfo[b, m] - np.floor(Cfo[b, m])
        assert abs(frac - 0.5) <= 1e-12 * Cfo[b, m] + 1e-9, (b, m, Cfo[b, m])
        if Cfg is not None:
            assert abs(Cfg[b, m] - Cfo[b, m]) <= 1e-12 * Cfo[b, m]
    return len(mism[0])


@pytest.fixture(scope="module")
def large():
    """The largest single-GPU instance (4,000 bases, 10,000 hospitals,
    100,000 missions) and the oracle's FP64 / int32 tables of it."""
    inst = synth.workload_instance("large")
    Co, Cfo = oracle.cost_table(inst.bases, inst.missions, want_cf=True)
    yield inst, Co, Cfo
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_cost_table_full_size(large):
    """The whole 4,000 x 100,000 table on the GPU, direct and indexed forms:
    the indexed table (missions as hospital-id pairs) equals the direct one
    bit for bit (int32 and FP64); every FP64 entry is within 1e-12 of the
    oracle's, and every int32 entry that differs from the oracle's sits on a
    rounding boundary."""
    inst, Co, Cfo = large
    B, M = Co.shape
    Cg, Cfg = fs.build_cost_table(to_dev(inst.bases), to_dev(inst.missions), want_cf=True)
    Ci, Cfi = fs.build_cost_table_indexed(to_dev(inst.bases), to_dev(inst.hospitals),
                                          to_dev(inst.mission_ph), want_cf=True)
    assert torch.equal(Cg, Ci)
    assert torch.equal(Cfg.contiguous().view(torch.int64), Cfi.contiguous().view(torch.int64))
    del Ci, Cfi
    n_mism = 0
    worst = 0.0
    for b0 in range(0, B, 500):
        cg = Cg[b0:b0 + 500].cpu().numpy()
        cfg = Cfg[b0:b0 + 500].cpu().numpy()
        cfo = Cfo[b0:b0 + 500]
        worst = max(worst, float((np.abs(cfg - cfo) / cfo).max()))
        n_mism += explain_mismatches(cg, Co[b0:b0 + 500], cfo, cfg)
    assert worst <= 1e-12, worst
    print(f"full-size table: max relative FP64 difference {worst:.3g}, "
          f"{n_mism} int32 entries on a rounding boundary", flush=True)
    del Cg, Cfg
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ rank (A1)


@pytest.mark.parametrize("ldc_pad", [0, 4, 1])
def test_rank_matches_oracle(ldc_pad):
    rng = np.random.default_rng(2 + ldc_pad)
    cases = [oracle_table(synth.workload_instance("small")), oracle_table(synth.workload_instance("medium"))]
    cases += [rng.integers(0, 3, size=(300, 257)).astype(np.int32)]   # many equal sums
    for C in cases:
        B, M = C.shape
        ldc = M + ldc_pad
        Cd = padded_table(C, ldc)
        for K in (1, 5, min(B, 30), B):
            op, order, sums = fs.rank_bases(Cd, K, M=M)
            o_open, o_order, o_sums = oracle.rank_bases(C, K)
            assert np.array_equal(sums.cpu().numpy(), o_sums)
            assert np.array_equal(order.cpu().numpy(), o_order)
            assert np.array_equal(op.cpu().numpy(), o_open)


# ------------------------------------------------------------------ move scores (A2, A3)


def check_scores(C, S, R, ldc=None):
    B, M = C.shape
    Cd = padded_table(C, ldc or M)
    cov, dist = fs.move_scores(Cd, torch.tensor(S, dtype=torch.int32), R, M=M)
    ocov, odist = oracle.move_scores(C, np.array(S, dtype=np.int32), R)
    assert np.array_equal(cov.cpu().numpy(), ocov)
    assert np.array_equal(dist.cpu().numpy(), odist)


def test_move_scores_small_and_medium():
    for cfg in ("small", "medium"):
        c = synth.WORKLOADS[cfg]
        _, C = instance_and_table(cfg)
        S = oracle.rank_bases(C, c["K"])[0]
        check_scores(C, S.tolist(), c["R"])


# (rows per workgroup, mission chunks, loads in flight, non-temporal loads,
#  queued scoring, 1024-thread sweep workgroups, one mission per refresh thread)
GEOMETRIES = [(1, 1, 1, 1, 1, 0, 0), (2, 3, 2, 0, 0, 0, 1), (4, 1, 4, 1, 1, 0, 0),
              (8, 5, 1, 1, 1, 0, 1), (1, 7, 4, 0, 1, 1, 0), (2, 1, 4, 1, 1, 1, 1),
              (4, 2, 2, 1, 0, 0, 0), (1, 1, 2, 1, 0, 1, 1), (2, 2, 1, 1, 0, 1, 0),
              (4, 1, 1, 1, 0, 1, 1), (8, 1, 1, 0, 0, 1, 0), (16, 1, 1, 1, 0, 0, 0),
              (16, 3, 1, 0, 0, 1, 1), (8, 2, 1, 1, 0, 0, 1)]


@pytest.mark.parametrize("J,split,U,nt,q,w,rw", GEOMETRIES)
def test_move_scores_launch_geometries(J, split, U, nt, q, w, rw):
    inst = synth.make_instance(seed=31, B=90, H=200, M=4103)
    C = oracle_table(inst)
    rng = np.random.default_rng(J * 10 + split)
    S = rng.choice(90, 11, replace=False).tolist()
    with env(FS_SWEEP_J=J, FS_SWEEP_SPLIT=split, FS_SWEEP_U=U, FS_SWEEP_NT=nt,
             FS_SWEEP_QUEUE=q, FS_SWEEP_WIDE=w, FS_REFRESH_WIDE=rw):
        check_scores(C, S, 1_000_000, ldc=4104)   # 16-byte rows
        check_scores(C, S, 1_000_000)             # 4-byte rows (ldc % 4 != 0)


def test_move_scores_random_small():
    rng = np.random.default_rng(41)
    for trial in range(40):
        B = int(rng.integers(2, 40))
        M = int(rng.integers(1, 300))
        K = int(rng.integers(1, B))
        C = rng.integers(1, 2000, size=(B, M)).astype(np.int32)
        if trial % 3 == 0:
            C = rng.integers(1, 6, size=(B, M)).astype(np.int32)    # ties everywhere
        R = int(rng.integers(0, 2100))
        S = rng.choice(B, K, replace=False).tolist()
        check_scores(C, S, R, ldc=M + int(rng.integers(0, 5)))


# ------------------------------------------------------------------ tabu search (A4-A6)


def run_both(C, K, R, T, N, mode=0, init=None, ldc=None):
    B, M = C.shape
    Cd = padded_table(C, ldc or M)
    init_d = None if init is None else torch.tensor(init, dtype=torch.int32)
    g = fs.tabu_solve(Cd, K, R, T, N, mode=mode, init_open=init_d, M=M)
    o = oracle.tabu(C, K, R, T, N, mode=mode, init_open=init)
    return g, o


def assert_same_result(g, o, C, R):
    assert np.array_equal(g.best_open.cpu().numpy(), o.best_open)
    assert (g.coverage, g.distance, g.best_iter) == (o.coverage, o.distance, o.best_iter)
    if g.trace is not None:
        assert_trace_equal(g.trace, o)
    if g.assign is not None:
        assert np.array_equal(g.assign.cpu().numpy(), oracle.assign(C, o.best_open, R))


@pytest.mark.parametrize("cfg", ["small", "medium"])
def test_tabu_full_trace_configs(cfg):
    c = synth.WORKLOADS[cfg]
    _, C = instance_and_table(cfg)
    g, o = run_both(C, c["K"], c["R"], c["T"], c["N"], ldc=(c["M"] + 3) // 4 * 4)
    assert_same_result(g, o, C, c["R"])


@pytest.mark.parametrize("split4", [0, 1])
def test_refresh_forms_medium(split4):
    # the refresh in 64-mission workgroups and in 1024-thread workgroups of
    # 256 missions (four waves per 64 missions splitting the open slots)
    c = synth.WORKLOADS["medium"]
    _, C = instance_and_table("medium")
    with env(FS_REFRESH_SPLIT4=split4, FS_REFRESH_WIDE=0):
        g, o = run_both(C, c["K"], c["R"], c["T"], 120)
    assert_same_result(g, o, C, c["R"])


@pytest.mark.parametrize("persist,tab", [(0, 1), (1, 1), (1, 0)])
@pytest.mark.parametrize("mode", [0, 1])
def test_persistent_search_small_and_random(persist, tab, mode):
    # the whole search in one workgroup per instance (persistent launch; the
    # table in LDS or in device memory) against the oracle, and the
    # per-iteration launches, on the small workload and random tables with
    # ties and ragged mission counts
    c = synth.WORKLOADS["small"]
    _, C = instance_and_table("small")
    with env(FS_PERSIST=persist, FS_PERSIST_TAB=tab):
        g, o = run_both(C, c["K"], c["R"], c["T"], c["N"], mode=mode, ldc=(c["M"] + 3) // 4 * 4)
    assert_same_result(g, o, C, c["R"])
    rng = np.random.default_rng(900 + 10 * persist + 100 * tab + mode)
    for trial in range(12):
        B = int(rng.integers(2, 90))
        K = int(rng.integers(1, min(B, 64) + 1))
        M = int(rng.integers(1, 3000))
        C = rng.integers(0, 400, size=(B, M)).astype(np.int32)
        R = int(rng.integers(0, 420))
        init = None if trial % 3 == 0 else np.sort(rng.choice(B, K, replace=False)).astype(np.int32)
        with env(FS_PERSIST=persist, FS_PERSIST_TAB=tab):
            g, o = run_both(C, K, R, int(rng.integers(0, 9)), int(rng.integers(1, 60)),
                            mode=mode, init=init, ldc=(M + 3) // 4 * 4)
        assert_same_result(g, o, C, R)


@pytest.mark.parametrize("cfg", ["small", "medium"])
def test_local_search_configs(cfg):
    c = synth.WORKLOADS[cfg]
    _, C = instance_and_table(cfg)
    g, o = run_both(C, c["K"], c["R"], c["T"], c["N"], mode=1)
    assert_same_result(g, o, C, c["R"])


def test_tabu_golden_fixtures_on_gpu():
    import json
    gdir = os.path.join(os.path.dirname(__file__), "golden")
    for name in ("tabu_aspiration.json", "tabu_coverage.json", "tabu_zero_range.json"):
        fx = json.load(open(os.path.join(gdir, name)))
        C = np.array(fx["C"], dtype=np.int32)
        for run in fx["runs"]:
            g, o = run_both(C, fx["K"], fx["R"], run["T"], run["N"], mode=run["mode"],
                            init=fx.get("init_open"))
            assert g.best_open.cpu().numpy().tolist() == run["best_open"]
            assert (g.coverage, g.distance, g.best_iter) == (run["coverage"], run["distance"],
                                                            run["best_iter"])
            assert g.trace["out_base"].tolist() == run["out"]
            assert g.trace["in_base"].tolist() == run["in"]
            assert g.trace["cur_dist"].tolist() == run["cur_dist"]


def test_tabu_random_instances():
    rng = np.random.default_rng(51)
    for trial in range(30):
        B = int(rng.integers(2, 60))
        M = int(rng.integers(1, 700))
        K = int(rng.integers(1, B + 1))
        C = rng.integers(1, 5000, size=(B, M)).astype(np.int32)
        if trial % 4 == 0:
            C = rng.integers(1, 8, size=(B, M)).astype(np.int32)
        R = int(rng.integers(0, 5200))
        T = int(rng.integers(0, 12))
        N = int(rng.integers(0, 40))
        mode = int(trial % 5 == 0)
        init = None if trial % 2 else rng.choice(B, K, replace=False).tolist()
        g, o = run_both(C, K, R, T, N, mode=mode, init=init, ldc=M + int(rng.integers(0, 4)))
        assert_same_result(g, o, C, R)


@pytest.mark.parametrize("J", [1, 2])
def test_local_search_stop_and_geometry(J):
    """Local search stops early; the remaining records are no-move records,
    with and without the split-mission scoring kernel."""
    c = synth.WORKLOADS["small"]
    _, C = instance_and_table("small")
    for split in (1, 2):
        with env(FS_SWEEP_J=J, FS_SWEEP_SPLIT=split):
            g, o = run_both(C, c["K"], c["R"], c["T"], 40, mode=1)
        assert_same_result(g, o, C, c["R"])
        assert g.trace["moved"][-1] == 0


def test_special_cases():
    rng = np.random.default_rng(61)
    C = rng.integers(1, 100, size=(12, 50)).astype(np.int32)
    # every base open: no move, value of the full set
    g, o = run_both(C, 12, 80, 3, 6)
    assert_same_result(g, o, C, 80)
    assert g.trace["moved"].sum() == 0
    # zero range: nothing covered
    g, o = run_both(C, 3, 0, 2, 9)
    assert_same_result(g, o, C, 0)
    assert g.coverage == 0 and g.distance == 0
    # one vehicle
    g, o = run_both(C, 1, 90, 4, 5)
    assert_same_result(g, o, C, 90)
    # no iterations
    g, o = run_both(C, 4, 90, 4, 0)
    assert_same_result(g, o, C, 90)


def test_plans_are_bit_identical():
    """The result does not depend on the sweep's launch geometry."""
    c = synth.WORKLOADS["medium"]
    _, C = instance_and_table("medium")
    Cd = padded_table(C, c["M"])
    ref = fs.tabu_solve(Cd, c["K"], c["R"], c["T"], 60)
    for J, split, U, nt, q, w, rw in ((1, 1, 1, 1, 1, 0, 0), (2, 4, 2, 0, 0, 0, 1),
                                      (4, 9, 4, 1, 1, 0, 0), (8, 2, 1, 0, 1, 0, 1),
                                      (4, 1, 2, 1, 0, 0, 1), (1, 3, 4, 1, 1, 1, 0),
                                      (1, 1, 4, 0, 0, 1, 1), (2, 1, 2, 1, 1, 1, 0),
                                      (4, 1, 1, 1, 0, 1, 1)):
        with env(FS_SWEEP_J=J, FS_SWEEP_SPLIT=split, FS_SWEEP_U=U, FS_SWEEP_NT=nt,
                 FS_SWEEP_QUEUE=q, FS_SWEEP_WIDE=w, FS_REFRESH_WIDE=rw):
            g = fs.tabu_solve(Cd, c["K"], c["R"], c["T"], 60)
        assert np.array_equal(g.trace, ref.trace)
        assert np.array_equal(g.best_open.cpu().numpy(), ref.best_open.cpu().numpy())


@pytest.fixture(scope="module")
def large_oracle_run(large):
    """The oracle's whole 200-iteration Tabu search on the largest instance
    (the shared int32 table is the oracle's)."""
    _, Co, _ = large
    c = synth.WORKLOADS["large"]
    return oracle.tabu(Co, c["K"], c["R"], c["T"], c["N"])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("sparse", [1, 0])
def test_full_size_trajectory(large, large_oracle_run, sparse):
    """Largest single-GPU instance (4,000 bases, 100,000 missions, 64
    vehicles, 200 iterations): every trace record, the best placement, its
    value and the mission assignment equal the oracle's, with the sparse
    sweep (the default at this size) and with the dense sweep."""
    _, Co, _ = large
    c = synth.WORKLOADS["large"]
    o = large_oracle_run
    Cd = to_dev(Co)
    with env(FS_SPARSE=sparse):
        g = fs.tabu_solve(Cd, c["K"], c["R"], c["T"], c["N"])
    assert_trace_equal(g.trace, o)
    assert np.array_equal(g.best_open.cpu().numpy(), o.best_open)
    assert (g.coverage, g.distance, g.best_iter) == (o.coverage, o.distance, o.best_iter)
    assert np.array_equal(g.assign.cpu().numpy(), oracle.assign(Co, o.best_open, c["R"]))
    del Cd
    torch.cuda.empty_cache()


def test_built_table_carries_its_mission_count():
    """build_cost_table returns a (B, M) view of rows padded to a multiple of
    4; every call that takes it reads M and the pitch from the view, so the
    padding (uninitialised memory) never counts as missions."""
    inst = synth.make_instance(seed=41, B=60, H=150, M=1001)
    C, _ = fs.build_cost_table(to_dev(inst.bases), to_dev(inst.missions))
    assert tuple(C.shape) == (60, 1001) and C.stride(0) == 1004
    Ch = C.cpu().numpy()
    K, R, T, N = 7, 1_100_000, 5, 40
    g = fs.tabu_solve(C, K, R, T, N)
    o = oracle.tabu(Ch, K, R, T, N)
    assert_same_result(g, o, Ch, R)
    op, _, sums = fs.rank_bases(C, K)
    assert np.array_equal(op.cpu().numpy(), oracle.rank_bases(Ch, K)[0])
    assert np.array_equal(sums.cpu().numpy(), Ch.astype(np.int64).sum(axis=1))
    cov, dist = fs.move_scores(C, op, R)
    ocov, odist = oracle.move_scores(Ch, oracle.rank_bases(Ch, K)[0], R)
    assert np.array_equal(cov.cpu().numpy(), ocov) and np.array_equal(dist.cpu().numpy(), odist)
    b = fs.tabu_solve_batch([dict(C=C, K=K, range_m=R)], T, N)[0]
    assert np.array_equal(b.best_open.cpu().numpy(), o.best_open)
    assert (b.coverage, b.distance, b.best_iter) == (o.coverage, o.distance, o.best_iter)


def test_invalid_arguments_leave_outputs_untouched():
    C = np.ones((5, 8), dtype=np.int32)
    Cd = to_dev(C)
    with pytest.raises(fs.FleetstageError) as e:
        fs.tabu_solve(Cd, 6, 10, 1, 3)
    assert e.value.status == fs.FS_E_INVALID
    with pytest.raises(fs.FleetstageError) as e:
        fs.tabu_solve(Cd, 2, 10, 1, 3, init_open=torch.tensor([1, 1], dtype=torch.int32))
    assert e.value.status == fs.FS_E_INVALID
    with pytest.raises(fs.FleetstageError) as e:
        fs.tabu_solve(Cd, 2, -1, 1, 3)
    assert e.value.status == fs.FS_E_INVALID
