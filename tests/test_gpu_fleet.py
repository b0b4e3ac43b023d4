"""GPU parity of the heterogeneous fleet (rotary- and fixed-wing vehicles,
aerodromes and heliports, rotary-only missions; Section 3, Eq. 4-10, the typed
ranking of Algorithm 1 and the relocation search): the HIP path through the C
ABI against the CPU oracle on the same seeded inputs, bit for bit."""

import os

import numpy as np
import pytest
import torch

import oracle
from paper_2001_05291_amd import synth

pytestmark = pytest.mark.gpu

from gpu_util import assert_trace_equal, oracle_table, padded_table, to_dev  # noqa: E402

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


def typed_instance(seed, B, H, M, **kw):
    inst = synth.make_instance(seed=seed, B=B, H=H, M=M)
    hel, rho = synth.fleet_flags(seed, B, inst.mission_ph, H, **kw)
    return oracle_table(inst), hel, rho


def random_placement(rng, B, K_r, K_f, hel):
    """K_r rotary-wing vehicles anywhere, K_f fixed-wing ones on aerodromes."""
    aero = np.flatnonzero(hel == 0)
    fixed = rng.choice(aero, K_f, replace=False)
    rest = np.setdiff1d(np.arange(B), fixed)
    rot = rng.choice(rest, K_r, replace=False)
    S = np.concatenate([rot, fixed]).astype(np.int32)
    types = np.array([1] * K_r + [0] * K_f, dtype=np.int32)
    perm = rng.permutation(K_r + K_f)
    return S[perm], types[perm]


def check_move_scores(C, hel, rho, S, types, R, ldc=None):
    B, M = C.shape
    K_r, K_f = int(types.sum()), int(len(types) - types.sum())
    Cd = padded_table(C, ldc or M)
    cov, dist = fs.fleet_move_scores(Cd, K_r, K_f, hel, rho, S, types, R, M=M)
    ocov, odist = oracle.fleet_move_scores(C, S, types, hel, rho, R)
    assert np.array_equal(cov.cpu().numpy(), ocov)
    assert np.array_equal(dist.cpu().numpy(), odist)


def test_fleet_move_scores_random_placements():
    rng = np.random.default_rng(71)
    C, hel, rho = typed_instance(3, B=70, H=160, M=1203)
    for K_r, K_f in [(4, 3), (7, 0), (0, 6), (1, 1), (10, 12)]:
        S, types = random_placement(rng, 70, K_r, K_f, hel)
        check_move_scores(C, hel, rho, S, types, 1_000_000, ldc=1204)
        check_move_scores(C, hel, rho, S, types, 800_000)


# (rows per workgroup, mission chunks, non-temporal loads, queued scoring,
#  1024-thread sweep workgroups, one mission per refresh thread); typed
#  sweeps keep one load in flight
GEOMETRIES = [(1, 1, 1, 1, 0, 0), (2, 3, 0, 0, 0, 1), (4, 1, 1, 1, 0, 0), (8, 5, 1, 1, 0, 1),
              (16, 2, 1, 0, 0, 0),
              (1, 7, 0, 1, 1, 1), (4, 2, 1, 0, 0, 0), (1, 1, 1, 0, 1, 0), (2, 1, 0, 1, 1, 1),
              (4, 1, 1, 0, 1, 0), (8, 1, 0, 0, 1, 1)]


@pytest.mark.parametrize("J,split,nt,q,w,rw", GEOMETRIES)
def test_fleet_move_scores_launch_geometries(J, split, nt, q, w, rw):
    C, hel, rho = typed_instance(31, B=90, H=200, M=4103)
    rng = np.random.default_rng(J * 10 + split)
    S, types = random_placement(rng, 90, 6, 5, hel)
    with env(FS_SWEEP_J=J, FS_SWEEP_SPLIT=split, FS_SWEEP_NT=nt, FS_SWEEP_QUEUE=q,
             FS_SWEEP_WIDE=w, FS_REFRESH_WIDE=rw):
        check_move_scores(C, hel, rho, S, types, 1_000_000, ldc=4104)   # 16-byte rows
        check_move_scores(C, hel, rho, S, types, 1_000_000)             # 4-byte rows


def test_fleet_move_scores_ties_and_small_tables():
    rng = np.random.default_rng(73)
    for trial in range(30):
        B = int(rng.integers(3, 40))
        M = int(rng.integers(1, 300))
        hel = (rng.random(B) < 0.4).astype(np.int32)
        rho = (rng.random(M) < 0.3).astype(np.int32)
        aero = int((hel == 0).sum())
        if aero == 0:
            continue
        K_f = int(rng.integers(0, min(aero, B - 1) + 1))
        K_r = int(rng.integers(0, B - K_f))
        if K_r + K_f == 0:
            K_r = 1
        hi = 6 if trial % 3 == 0 else 2000   # ties everywhere
        C = rng.integers(1, hi, size=(B, M)).astype(np.int32)
        R = int(rng.integers(0, hi + 100))
        S, types = random_placement(rng, B, K_r, K_f, hel)
        check_move_scores(C, hel, rho, S, types, R, ldc=M + int(rng.integers(0, 5)))


def run_both(C, hel, rho, K_r, K_f, R, T, N, mode=0, init=None, ldc=None):
    B, M = C.shape
    Cd = padded_table(C, ldc or M)
    S0 = r0 = None
    if init is not None:
        S0, r0 = init
    g = fs.fleet_solve(Cd, K_r, K_f, hel, rho, R, T, N, mode=mode, init_open=S0,
                       init_rotary=r0, M=M)
    o = oracle.fleet_tabu(C, K_r, K_f, hel, rho if rho is not None else np.zeros(M, np.int32),
                          R, T, N, mode=mode, init_open=S0, init_rot=r0)
    return g, o


def assert_same(g, o, C, rho, R):
    assert np.array_equal(g.best_open.cpu().numpy(), o.best_open)
    assert np.array_equal(g.best_rotary.cpu().numpy(), o.best_rot)
    assert (g.coverage, g.distance, g.best_iter) == (o.coverage, o.distance, o.best_iter)
    assert_trace_equal(g.trace, o)
    rho = rho if rho is not None else np.zeros(C.shape[1], np.int32)
    assert np.array_equal(g.assign.cpu().numpy(),
                          oracle.fleet_assign(C, o.best_open, o.best_rot, rho, R))


@pytest.mark.parametrize("mode", [0, 1])
def test_fleet_solve_full_trace(mode):
    C, hel, rho = typed_instance(5, B=120, H=300, M=2500)
    K_r, K_f = synth.fleet_split(14)
    g, o = run_both(C, hel, rho, K_r, K_f, 950_000, 7, 40, mode=mode, ldc=2500)
    assert_same(g, o, C, rho, 950_000)


def test_fleet_solve_given_placement_and_geometries():
    C, hel, rho = typed_instance(9, B=80, H=200, M=3001)
    rng = np.random.default_rng(9)
    S, types = random_placement(rng, 80, 5, 4, hel)
    for J, split, q, w in ((1, 1, 1, 1), (2, 3, 0, 0), (4, 1, 0, 1), (8, 2, 1, 0)):
        with env(FS_SWEEP_J=J, FS_SWEEP_SPLIT=split, FS_SWEEP_QUEUE=q, FS_SWEEP_WIDE=w):
            g, o = run_both(C, hel, rho, 5, 4, 900_000, 5, 30, init=(S, types), ldc=3004)
        assert_same(g, o, C, rho, 900_000)


def test_fleet_solve_random_small():
    rng = np.random.default_rng(79)
    done = 0
    for trial in range(40):
        B = int(rng.integers(3, 45))
        M = int(rng.integers(1, 500))
        hel = (rng.random(B) < 0.4).astype(np.int32)
        rho = (rng.random(M) < 0.3).astype(np.int32) if trial % 5 else None
        aero = int((hel == 0).sum())
        K_f = int(rng.integers(0, min(aero, B - 1) + 1))
        K_r = int(rng.integers(0 if K_f else 1, B - K_f + 1))
        if K_r + K_f > B or aero + min(int(hel.sum()), K_r) < K_r + K_f:
            continue
        hi = 8 if trial % 4 == 0 else 5000
        C = rng.integers(1, hi, size=(B, M)).astype(np.int32)
        R = int(rng.integers(0, hi + 200))
        T = int(rng.integers(0, 10))
        N = int(rng.integers(0, 35))
        mode = int(trial % 6 == 0)
        init = None if trial % 2 else random_placement(rng, B, K_r, K_f, hel)
        g, o = run_both(C, hel, rho, K_r, K_f, R, T, N, mode=mode, init=init,
                        ldc=M + int(rng.integers(0, 4)))
        assert_same(g, o, C, rho, R)
        done += 1
    assert done >= 20


def test_homogeneous_fleet_equals_plain_search():
    """No heliport and no rotary-only mission: the typed search is the plain
    one, whatever the split of the fleet into types."""
    inst = synth.workload_instance("small")
    c = synth.WORKLOADS["small"]
    C = oracle_table(inst)
    Cd = padded_table(C, (c["M"] + 3) // 4 * 4)[:, :c["M"]]
    hel = np.zeros(inst.B, np.int32)
    plain = fs.tabu_solve(Cd, c["K"], c["R"], c["T"], c["N"])
    for K_r in (c["K"], 2, 0):
        g = fs.fleet_solve(Cd, K_r, c["K"] - K_r, hel, None, c["R"], c["T"], c["N"])
        assert np.array_equal(g.best_open.cpu().numpy(), plain.best_open.cpu().numpy())
        assert (g.coverage, g.distance, g.best_iter) == (plain.coverage, plain.distance,
                                                        plain.best_iter)
        assert np.array_equal(g.trace, plain.trace)
        assert np.array_equal(g.assign.cpu().numpy(), plain.assign.cpu().numpy())


def test_only_fixed_wing_leaves_rotary_missions_uncovered():
    C, hel, rho = typed_instance(13, B=50, H=120, M=900)
    g, o = run_both(C, hel, rho, 0, 6, 1_500_000, 4, 15)
    assert_same(g, o, C, rho, 1_500_000)
    a = g.assign.cpu().numpy()
    assert np.all(a[rho == 1] == -1)


def test_fleet_invalid_arguments():
    C, hel, rho = typed_instance(17, B=12, H=40, M=60)
    Cd = to_dev(C)

    def bad(**kw):
        args = dict(K_r=2, K_f=2, heliport=hel, rotary_only=rho, range_m=1_000_000, tenure=2,
                    iterations=3)
        args.update(kw)
        with pytest.raises(fs.FleetstageError) as e:
            fs.fleet_solve(Cd, args["K_r"], args["K_f"], args["heliport"], args["rotary_only"],
                           args["range_m"], args["tenure"], args["iterations"],
                           init_open=args.get("init_open"), init_rotary=args.get("init_rotary"))
        assert e.value.status == fs.FS_E_INVALID
        return str(e.value)

    bad(K_r=-1)
    bad(K_r=0, K_f=0)
    aero = np.flatnonzero(hel == 0)
    heli = np.flatnonzero(hel == 1)
    assert len(heli) >= 1 and len(aero) >= 3
    bad(K_r=0, K_f=len(aero) + 1)                         # too many fixed-wing vehicles
    S = np.array([heli[0], aero[0], aero[1], aero[2]], np.int32)
    bad(init_open=S, init_rotary=np.array([0, 1, 1, 0], np.int32))   # fixed-wing on a heliport
    bad(init_open=S, init_rotary=np.array([1, 1, 1, 0], np.int32))   # three rotary-wing
    bad(init_open=S)                                                # types missing
    with pytest.raises(ValueError):
        fs.fleet_solve(Cd, 2, 2, hel[:5], rho, 1_000_000, 2, 3)
