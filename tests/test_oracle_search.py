"""Pins of the oracle's base ranking (Algorithm 1), move scores (the checks of
Algorithms 2-3) and Tabu / local search (Algorithm 3 / 2) against hand-derived
fixtures, brute force, special cases and invariants.  CPU only."""

import itertools
import json
import os

import numpy as np
import pytest

import oracle
from paper_2001_05291_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def brute_value(C, S, R):
    """Value of a placement by direct enumeration: per mission, the nearest
    open base; covered when within R."""
    cov, dist = 0, 0
    for m in range(C.shape[1]):
        v = min(int(C[s, m]) for s in S)
        if v <= R:
            cov += 1
            dist += v
    return cov, dist


def key(cov, dist):
    """Total order used for 'better': more coverage, then less distance."""
    return (-cov, dist)


def random_C(rng, B, M, lo=1, hi=60):
    return rng.integers(lo, hi, size=(B, M)).astype(np.int32)


# ---------------------------------------------------------------- rank


def test_rank_matches_textbook_sort():
    rng = np.random.default_rng(3)
    for _ in range(30):
        B, M = rng.integers(2, 40), rng.integers(1, 30)
        C = random_C(rng, B, M, 0, 4)          # many equal row sums
        K = int(rng.integers(1, B + 1))
        op, order, sums = oracle.rank_bases(C, K)
        ref_sums = C.astype(np.int64).sum(axis=1)
        assert np.array_equal(sums, ref_sums)
        ref_order = np.lexsort((np.arange(B), ref_sums))[:K]
        assert np.array_equal(order, ref_order)
        assert np.array_equal(op, np.sort(ref_order))


def test_rank_golden():
    for name in ("tabu_aspiration.json", "tabu_coverage.json"):
        g = load(name)
        C = np.array(g["C"], dtype=np.int32)
        op, order, sums = oracle.rank_bases(C, g["K"])
        assert op.tolist() == g["rank"]["open"]
        assert order.tolist() == g["rank"]["order"]
        assert sums.tolist() == g["rank"]["row_sums"]


# ---------------------------------------------------------------- value / scores


def test_placement_value_brute_force():
    rng = np.random.default_rng(4)
    for _ in range(40):
        B, M = int(rng.integers(2, 10)), int(rng.integers(1, 12))
        C = random_C(rng, B, M)
        K = int(rng.integers(1, B + 1))
        S = rng.choice(B, K, replace=False).astype(np.int32)
        R = int(rng.integers(0, 70))
        assert oracle.placement_value(C, S, R) == brute_value(C, S, R)


def test_move_scores_equal_recount_of_every_move():
    rng = np.random.default_rng(5)
    for trial in range(25):
        B, M = int(rng.integers(3, 14)), int(rng.integers(1, 40))
        C = random_C(rng, B, M)
        K = int(rng.integers(1, B))
        S = rng.choice(B, K, replace=False).astype(np.int32)
        R = int(rng.integers(0, 70))
        cov, dist = oracle.move_scores(C, S, R)
        for k, i in enumerate(S):
            for j in range(B):
                if j in S:
                    assert cov[k, j] == -1 and dist[k, j] == -1
                    continue
                T = [s for s in S if s != i] + [j]
                assert (cov[k, j], dist[k, j]) == brute_value(C, T, R), (trial, k, j)


def test_move_scores_golden():
    g = load("tabu_coverage.json")
    C = np.array(g["C"], dtype=np.int32)
    cov, dist = oracle.move_scores(C, np.array(g["move_scores_from"]), g["R"])
    assert cov.tolist() == g["move_cov"]
    assert dist.tolist() == g["move_dist"]
    assert oracle.placement_value(C, g["rank"]["open"], g["R"]) == tuple(g["value_of_rank"])


def test_assign_invariants_and_golden():
    g = load("tabu_coverage.json")
    C = np.array(g["C"], dtype=np.int32)
    assert oracle.assign(C, g["assign_of"], g["R"]).tolist() == g["assign"]
    rng = np.random.default_rng(6)
    for _ in range(30):
        B, M = int(rng.integers(2, 12)), int(rng.integers(1, 30))
        C = random_C(rng, B, M, 1, 8)          # many ties between bases
        K = int(rng.integers(1, B + 1))
        S = rng.choice(B, K, replace=False).astype(np.int32)
        R = int(rng.integers(0, 9))
        a = oracle.assign(C, S, R)
        cov, dist = oracle.placement_value(C, S, R)
        assert cov == int((a >= 0).sum())
        assert dist == int(sum(int(C[a[m], m]) for m in range(M) if a[m] >= 0))
        for m in range(M):
            best = min(int(C[s, m]) for s in S)
            if a[m] >= 0:
                assert C[a[m], m] == best <= R
                assert a[m] == min(s for s in S if C[s, m] == best)
            else:
                assert best > R


# ---------------------------------------------------------------- optimum


def test_brute_optimum_matches_itertools():
    rng = np.random.default_rng(7)
    for _ in range(20):
        B, M = int(rng.integers(2, 9)), int(rng.integers(1, 10))
        C = random_C(rng, B, M)
        K = int(rng.integers(1, B + 1))
        R = int(rng.integers(10, 70))
        best, cov, dist, n = oracle.brute_optimum(C, K, R)
        combos = list(itertools.combinations(range(B), K))
        assert n == len(combos)
        vals = [brute_value(C, c, R) for c in combos]
        top = min(range(len(combos)), key=lambda x: key(*vals[x]))
        assert (cov, dist) == vals[top]
        assert tuple(best.tolist()) == combos[top]


# ---------------------------------------------------------------- tabu: fixtures


@pytest.mark.parametrize("name", ["tabu_aspiration.json", "tabu_coverage.json",
                                  "tabu_zero_range.json"])
def test_tabu_golden(name):
    g = load(name)
    C = np.array(g["C"], dtype=np.int32)
    init = g.get("init_open")
    for run in g["runs"]:
        r = oracle.tabu(C, g["K"], g["R"], run["T"], run["N"], mode=run["mode"], init_open=init)
        assert r.best_open.tolist() == run["best_open"]
        assert (r.coverage, r.distance, r.best_iter) == (run["coverage"], run["distance"],
                                                        run["best_iter"])
        assert r.out_base.tolist() == run["out"]
        assert r.in_base.tolist() == run["in"]
        assert r.moved.tolist() == run["moved"]
        assert r.cur_cov.tolist() == run["cur_cov"]
        assert r.cur_dist.tolist() == run["cur_dist"]
        assert r.best_cov.tolist() == run["best_cov"]
        assert r.best_dist.tolist() == run["best_dist"]
    if "optimum" in g:
        best, cov, dist, n = oracle.brute_optimum(C, g["K"], g["R"])
        assert best.tolist() == g["optimum"]["open"]
        assert (cov, dist, n) == (g["optimum"]["coverage"], g["optimum"]["distance"],
                                  g["optimum"]["placements"])


# ---------------------------------------------------------------- tabu: invariants


def replay_check(C, K, R, init, res, N):
    """Replays the reported moves and checks every record against a recount."""
    S = list(init)
    cur = brute_value(C, S, R)
    best = cur
    best_S = sorted(S)
    best_iter = 0
    for t in range(N):
        if res.moved[t]:
            i, j = int(res.out_base[t]), int(res.in_base[t])
            assert i in S and j not in S
            S[S.index(i)] = j
            cur = brute_value(C, S, R)
            if key(*cur) < key(*best):
                best, best_S, best_iter = cur, sorted(S), t + 1
        else:
            assert res.out_base[t] == -1 and res.in_base[t] == -1
        assert (res.cur_cov[t], res.cur_dist[t]) == cur
        assert (res.best_cov[t], res.best_dist[t]) == best
    assert res.best_open.tolist() == best_S
    assert (res.coverage, res.distance, res.best_iter) == (*best, best_iter)
    assert res.coverage <= C.shape[1]


def test_tabu_invariants_random():
    rng = np.random.default_rng(8)
    for trial in range(30):
        B, M = int(rng.integers(3, 11)), int(rng.integers(2, 25))
        C = random_C(rng, B, M, 1, 40)
        K = int(rng.integers(1, B))
        R = int(rng.integers(5, 45))
        T = int(rng.integers(0, 5))
        N = int(rng.integers(1, 15))
        tabu = oracle.tabu(C, K, R, T, N, mode=0)
        ls = oracle.tabu(C, K, R, T, N, mode=1)
        init = oracle.rank_bases(C, K)[0]
        replay_check(C, K, R, init, tabu, N)
        replay_check(C, K, R, init, ls, N)
        # local search never beats the tabu search (same start, same tie-break)
        assert key(tabu.coverage, tabu.distance) <= key(ls.coverage, ls.distance)
        # the moves of local search are a prefix of the tabu trajectory
        n_ls = int(ls.moved.sum())
        assert np.all(ls.moved[:n_ls] == 1) and np.all(ls.moved[n_ls:] == 0)
        assert np.array_equal(ls.out_base[:n_ls], tabu.out_base[:n_ls])
        assert np.array_equal(ls.in_base[:n_ls], tabu.in_base[:n_ls])
        # neither beats the exhaustive optimum
        _, ocov, odist, _ = oracle.brute_optimum(C, K, R)
        assert key(ocov, odist) <= key(tabu.coverage, tabu.distance)


def test_local_search_ends_in_local_optimum():
    rng = np.random.default_rng(9)
    for _ in range(20):
        B, M = int(rng.integers(3, 10)), int(rng.integers(2, 20))
        C = random_C(rng, B, M, 1, 40)
        K = int(rng.integers(1, B))
        R = int(rng.integers(5, 45))
        ls = oracle.tabu(C, K, R, 0, 10 * B * B, mode=1)
        S = ls.best_open.tolist()
        here = brute_value(C, S, R)
        for i in S:
            for j in range(B):
                if j in S:
                    continue
                T = [s for s in S if s != i] + [j]
                assert key(*brute_value(C, T, R)) >= key(*here)


def test_all_bases_open_makes_no_move():
    rng = np.random.default_rng(10)
    C = random_C(rng, 6, 9)
    r = oracle.tabu(C, 6, 30, 3, 5)
    assert r.moved.tolist() == [0] * 5 and r.best_iter == 0
    assert r.best_open.tolist() == list(range(6))
    assert (r.coverage, r.distance) == brute_value(C, range(6), 30)


def test_zero_range_scores_nothing():
    rng = np.random.default_rng(11)
    C = random_C(rng, 7, 10, 1, 50)
    cov, dist = oracle.move_scores(C, np.array([1, 4]), 0)
    closed = [j for j in range(7) if j not in (1, 4)]
    assert np.all(cov[:, closed] == 0) and np.all(dist[:, closed] == 0)


def test_single_vehicle_finds_best_single_base():
    rng = np.random.default_rng(12)
    for _ in range(20):
        B, M = int(rng.integers(2, 15)), int(rng.integers(1, 20))
        C = random_C(rng, B, M, 1, 40)
        R = int(rng.integers(5, 45))
        T = int(rng.integers(0, 6))
        r = oracle.tabu(C, 1, R, T, int(rng.integers(1, 6)))
        vals = [brute_value(C, [b], R) for b in range(B)]
        top = min(range(B), key=lambda b: key(*vals[b]))
        assert (r.coverage, r.distance) == vals[top]
        assert r.best_open.tolist() == [top]


def test_zero_tenure_is_best_move_walk():
    """T = 0: every move is admissible, so each iteration takes the best swap
    of the current placement (a worsening one too)."""
    rng = np.random.default_rng(13)
    C = random_C(rng, 8, 15, 1, 40)
    K, R, N = 3, 30, 12
    r = oracle.tabu(C, K, R, 0, N)
    S = oracle.rank_bases(C, K)[0].tolist()
    for t in range(N):
        moves = []
        for i in S:
            for j in range(8):
                if j not in S:
                    T = [s for s in S if s != i] + [j]
                    moves.append((key(*brute_value(C, T, R)), i, j))
        _, i, j = min(moves)
        assert (r.out_base[t], r.in_base[t]) == (i, j)
        S[S.index(i)] = j


def test_tabu_thread_count_invariant():
    inst = synth.make_instance(seed=3, B=60, H=90, M=300)
    C, _ = oracle.cost_table(inst.bases, inst.missions, want_cf=False)
    n = oracle.get_threads()
    oracle.set_threads(1)
    a = oracle.tabu(C, 6, 1_100_000, 5, 20)
    oracle.set_threads(max(n, 2))
    b = oracle.tabu(C, 6, 1_100_000, 5, 20)
    oracle.set_threads(n)
    for f in ("best_open", "out_base", "in_base", "cur_cov", "cur_dist", "best_cov", "best_dist"):
        assert np.array_equal(getattr(a, f), getattr(b, f))


def test_small_workload_tabu_against_exhaustive_optimum():
    """Configuration 1 (40 bases, 200 missions, 5 vehicles, R = 1,200 km): the
    Tabu result never beats the optimum over all C(40,5) = 658,008 placements."""
    c = synth.WORKLOADS["small"]
    inst = synth.workload_instance("small")
    C, _ = oracle.cost_table(inst.bases, inst.missions, want_cf=False)
    r = oracle.tabu(C, c["K"], c["R"], c["T"], c["N"])
    best, cov, dist, n = oracle.brute_optimum(C, c["K"], c["R"])
    assert n == 658_008
    assert key(cov, dist) <= key(r.coverage, r.distance)
    assert r.coverage <= c["M"]
