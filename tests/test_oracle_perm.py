"""Pins of the permuted first-improvement searches of the oracle (Algorithms 2
and 3 with their random scan orders, Section 4.2-4.3) against the published
SplitMix64 outputs, brute-force recounts of every move at every step,
exhaustive optima and the relations between the variants.  CPU only."""

import itertools

import numpy as np
import pytest

import oracle


def value_np(C, S, R):
    v = C[np.asarray(S)].min(axis=0).astype(np.int64)
    cov = v <= R
    return int(cov.sum()), int(v[cov].sum())


def better(a, b):
    return a[0] > b[0] or (a[0] == b[0] and a[1] < b[1])


def random_table(seed, B=12, M=40, hi=1000):
    rng = np.random.default_rng(seed)
    return rng.integers(1, hi, size=(B, M)).astype(np.int32)


def test_mix64_matches_published_splitmix64_outputs():
    # the first four outputs of SplitMix64 from state 0 (state += GAMMA, then
    # the output function), as published with the generator
    g = 0x9E3779B97F4A7C15
    expected = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert [oracle.mix64((k * g) % 2**64) for k in range(1, 5)] == expected


def test_priorities_are_a_permutation_of_the_moves():
    B = 60
    for seed, p in [(0, 0), (5, 3), (2**63 + 11, 1)]:
        pis = {oracle.perm_priority(seed, p, B, i, j) for i in range(B) for j in range(B)}
        assert len(pis) == B * B
    # a pass and a seed each reorder the moves
    a = [oracle.perm_priority(1, 0, 20, i, 5) for i in range(20)]
    b = [oracle.perm_priority(1, 1, 20, i, 5) for i in range(20)]
    c = [oracle.perm_priority(2, 0, 20, i, 5) for i in range(20)]
    assert np.argsort(a).tolist() != np.argsort(b).tolist()
    assert np.argsort(a).tolist() != np.argsort(c).tolist()


def check_trajectory(C, K, R, T, mode, seed, res, S0):
    """Replays the trace and checks, at every record, the selection rule from
    a brute-force recount of every move of the current placement."""
    B = C.shape[0]
    S = list(S0)
    cur = value_np(C, S, R)
    tabu_until = np.zeros(B, dtype=np.int64)
    p, last, accepted, stopped = 0, None, False, False
    for t in range(1, len(res.moved) + 1):
        rec = t - 1
        # admissible improving moves after the last accepted one, by priority
        cands = []
        if not stopped:
            for k, i in enumerate(S):
                for j in range(B):
                    if j in S:
                        continue
                    pi = oracle.perm_priority(seed, p, B, i, j)
                    if last is not None and pi <= last:
                        continue
                    if mode == 3 and not (tabu_until[i] < t and tabu_until[j] < t):
                        continue
                    S2 = list(S)
                    S2[k] = j
                    v = value_np(C, S2, R)
                    if better(v, cur):
                        cands.append((pi, k, i, j, v))
        if res.moved[rec]:
            assert cands, f"move at record {rec} although no admissible improvement exists"
            pi, k, i, j, v = min(cands)
            assert (res.out_base[rec], res.in_base[rec]) == (i, j), rec
            S[k] = j
            cur = v
            tabu_until[i] = tabu_until[j] = t + T
            last, accepted = pi, True
        else:
            assert not cands, f"no move at record {rec} although {len(cands)} improve"
            if not stopped:
                if accepted:
                    p, last, accepted = p + 1, None, False
                else:
                    stopped = True
        assert (res.cur_cov[rec], res.cur_dist[rec]) == cur
        assert (res.best_cov[rec], res.best_dist[rec]) == cur
    assert value_np(C, res.best_open, R) == (res.coverage, res.distance) == cur
    return stopped, p


@pytest.mark.parametrize("mode", [2, 3])
def test_selection_rule_by_brute_force(mode):
    for seed in range(6):
        C = random_table(seed, B=11, M=35)
        if seed % 3 == 0:
            C = random_table(seed, B=11, M=35, hi=6)   # many equal values
        K, R, T, N = 3, 700 if seed % 3 else 5, 2, 40
        S0 = oracle.rank_bases(C, K)[0]
        res = oracle.perm_search(C, K, R, T, N, mode, seed * 7919)
        stopped, passes = check_trajectory(C, K, R, T, mode, seed * 7919, res, S0)
        assert passes == res.passes


def test_given_start_and_local_optimum_at_stop():
    rng = np.random.default_rng(3)
    for trial in range(6):
        C = random_table(100 + trial, B=10, M=30)
        K, R = 3, 650
        S0 = rng.choice(10, K, replace=False).astype(np.int32)
        res = oracle.perm_search(C, K, R, 0, 60, 2, trial, init_open=S0)
        stopped, _ = check_trajectory(C, K, R, 0, 2, trial, res, S0)
        assert stopped
        # no swap improves the final placement
        S = list(res.best_open)
        cur = value_np(C, S, R)
        for k in range(K):
            for j in range(10):
                if j not in S:
                    S2 = list(S)
                    S2[k] = j
                    assert not better(value_np(C, S2, R), cur)


def test_bounded_by_the_exhaustive_optimum():
    for seed in range(4):
        C = random_table(200 + seed, B=9, M=25)
        K, R = 3, 600
        best = max((value_np(C, list(S), R) for S in itertools.combinations(range(9), K)),
                   key=lambda v: (v[0], -v[1]))
        for mode in (2, 3):
            res = oracle.perm_search(C, K, R, 3, 50, mode, seed)
            assert (res.coverage, -res.distance) <= (best[0], -best[1])


def test_tabu_with_zero_tenure_is_the_local_search():
    for seed in range(5):
        C = random_table(300 + seed, B=13, M=45)
        a = oracle.perm_search(C, 4, 650, 0, 50, 2, seed)
        b = oracle.perm_search(C, 4, 650, 0, 50, 3, seed)
        for f in ("moved", "out_base", "in_base", "cur_cov", "cur_dist"):
            assert np.array_equal(getattr(a, f), getattr(b, f))


def test_seeds_vary_the_search_and_repeat_exactly():
    C = random_table(7, B=30, M=120)
    runs = [oracle.perm_search(C, 5, 600, 2, 80, 2, s) for s in range(8)]
    again = oracle.perm_search(C, 5, 600, 2, 80, 2, 3)
    assert np.array_equal(runs[3].in_base, again.in_base)
    assert len({tuple(r.in_base.tolist()) for r in runs}) > 1


def test_tabu_never_moves_a_tabu_base():
    C = random_table(11, B=25, M=90)
    T = 4
    res = oracle.perm_search(C, 5, 650, T, 80, 3, 99)
    last_move = {}
    for t in range(1, 81):
        rec = t - 1
        if res.moved[rec]:
            for b in (res.out_base[rec], res.in_base[rec]):
                assert t > last_move.get(int(b), -10**9) + T
                last_move[int(b)] = t
