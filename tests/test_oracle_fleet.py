"""Pins of the heterogeneous-fleet oracle (Section 3, Eq. 2-10) against
independent numpy recounts, exhaustive enumeration and the homogeneous oracle
it reduces to.  CPU only."""

import itertools

import numpy as np
import pytest

import oracle


def value_np(C, S, rot, rho, R):
    """Nearest compatible occupied base per mission, by numpy (independent)."""
    S = np.asarray(S)
    rot = np.asarray(rot).astype(bool)
    sub = C[S].astype(np.int64)                       # K x M
    any_min = sub.min(axis=0)
    rot_min = sub[rot].min(axis=0) if rot.any() else np.full(C.shape[1], np.iinfo(np.int64).max)
    v = np.where(np.asarray(rho).astype(bool), rot_min, any_min)
    cov = v <= R
    return int(cov.sum()), int(v[cov].sum())


def random_case(seed, B=14, M=40, hel_p=0.35, rho_p=0.3, lo=1, hi=900):
    rng = np.random.default_rng(seed)
    C = rng.integers(lo, hi, size=(B, M)).astype(np.int32)
    hel = (rng.random(B) < hel_p).astype(np.int32)
    rho = (rng.random(M) < rho_p).astype(np.int32)
    return C, hel, rho


def test_value_matches_numpy_recount():
    for seed in range(20):
        C, hel, rho = random_case(seed)
        rng = np.random.default_rng(100 + seed)
        S = rng.choice(C.shape[0], 5, replace=False)
        rot = (rng.random(5) < 0.5).astype(np.int32)
        R = int(rng.integers(200, 900))
        assert oracle.fleet_value(C, S, rot, rho, R) == value_np(C, S, rot, rho, R)


def test_move_scores_are_values_of_the_moved_placements():
    for seed in range(8):
        C, hel, rho = random_case(seed, B=12, M=30)
        rng = np.random.default_rng(200 + seed)
        S = rng.choice(12, 4, replace=False)
        rot = np.array([1, 0, 1, 0], dtype=np.int32)
        R = 700
        cov, dist = oracle.fleet_move_scores(C, S, rot, hel, rho, R)
        for k in range(4):
            for j in range(12):
                if j in S or (hel[j] and not rot[k]):
                    assert cov[k, j] == -1 and dist[k, j] == -1
                    continue
                S2 = S.copy()
                S2[k] = j
                assert (cov[k, j], dist[k, j]) == value_np(C, S2, rot, rho, R), (k, j)


def test_assign_invariants():
    C, hel, rho = random_case(3, B=16, M=60)
    S = np.array([1, 4, 9, 12])
    rot = np.array([1, 1, 0, 0], dtype=np.int32)
    R = 500
    a = oracle.fleet_assign(C, S, rot, rho, R)
    cov, dist = oracle.fleet_value(C, S, rot, rho, R)
    assert (a >= 0).sum() == cov
    assert sum(int(C[a[m], m]) for m in range(60) if a[m] >= 0) == dist
    for m in range(60):
        if a[m] >= 0:
            assert rot[list(S).index(a[m])] or not rho[m]   # a rotary-only mission flies rotary
            assert C[a[m], m] <= R


def test_rank_respects_heliport_cap_and_type_order():
    for seed in range(10):
        C, hel, rho = random_case(seed, B=20, M=30, hel_p=0.6)
        K_r, K_f = 3, 2
        if (1 - hel).sum() < K_f:
            continue
        S, rot = oracle.fleet_rank(C, K_r, K_f, hel)
        sums = C.astype(np.int64).sum(axis=1)
        # independent selection: walk bases by (sum, id), skip heliports past K_r
        order = np.lexsort((np.arange(20), sums))
        chosen, nh = [], 0
        for b in order:
            if hel[b] and nh >= K_r:
                continue
            chosen.append(int(b))
            nh += int(hel[b])
            if len(chosen) == K_r + K_f:
                break
        assert sorted(S.tolist()) == sorted(chosen)
        assert all(rot[k] == 1 for k in range(len(S)) if hel[S[k]])     # heliports: rotary
        assert int(rot.sum()) == K_r
        # aerodromes: rotary to the better-ranked ones
        aero = [b for b in chosen if not hel[b]]
        rot_aero = [int(rot[list(S).index(b)]) for b in aero]
        assert rot_aero == sorted(rot_aero, reverse=True)


def test_rank_rejects_a_fleet_the_bases_cannot_hold():
    C, _, _ = random_case(1, B=6, M=10)
    hel = np.array([1, 1, 1, 1, 1, 0], dtype=np.int32)
    with pytest.raises(ValueError):
        oracle.fleet_rank(C, 1, 2, hel)     # two fixed-wing, one aerodrome


def test_homogeneous_case_is_the_plain_model():
    """No heliport and no rotary-only mission: vehicle types do not matter and
    the typed search is the homogeneous one, move for move."""
    for seed, (K_r, K_f) in zip(range(6), [(4, 0), (2, 2), (0, 4), (3, 1), (1, 3), (4, 0)]):
        C, _, _ = random_case(seed, B=15, M=50)
        hel = np.zeros(15, dtype=np.int32)
        rho = np.zeros(50, dtype=np.int32)
        R = 600
        f = oracle.fleet_tabu(C, K_r, K_f, hel, rho, R, 3, 25)
        h = oracle.tabu(C, K_r + K_f, R, 3, 25)
        assert np.array_equal(f.best_open, h.best_open)
        assert (f.coverage, f.distance, f.best_iter) == (h.coverage, h.distance, h.best_iter)
        for a, b in zip((f.out_base, f.in_base, f.moved, f.cur_cov, f.cur_dist),
                        (h.out_base, h.in_base, h.moved, h.cur_cov, h.cur_dist)):
            assert np.array_equal(a, b)


def brute_np(C, K_r, K_f, hel, rho, R):
    B = C.shape[0]
    best = None
    for rset in itertools.combinations(range(B), K_r):
        rest = [b for b in range(B) if b not in rset and not hel[b]]
        for fset in itertools.combinations(rest, K_f):
            S = list(rset) + list(fset)
            rot = [1] * K_r + [0] * K_f
            v = value_np(C, S, rot, rho, R)
            if best is None or v[0] > best[0] or (v[0] == best[0] and v[1] < best[1]):
                best = v
    return best


def test_brute_optimum_matches_itertools():
    for seed in range(5):
        C, hel, rho = random_case(seed, B=9, M=25)
        if (1 - hel).sum() < 2:
            continue
        S, rot, cov, dist, n = oracle.fleet_brute_optimum(C, 2, 2, hel, rho, 600)
        assert (cov, dist) == brute_np(C, 2, 2, hel, rho, 600)
        assert value_np(C, S, rot, rho, 600) == (cov, dist)
        assert not any(hel[S[k]] and not rot[k] for k in range(4))


def replay(C, hel, rho, R, S0, rot0, res):
    """Re-applies every recorded move: each is a relocation to a free base the
    vehicle may use, and the recorded current value is the recount."""
    S = list(S0)
    rot = list(rot0)
    for t in range(len(res.moved)):
        if res.moved[t]:
            i, j = int(res.out_base[t]), int(res.in_base[t])
            k = S.index(i)
            assert j not in S
            assert not (hel[j] and not rot[k])
            S[k] = j
        assert (int(res.cur_cov[t]), int(res.cur_dist[t])) == value_np(C, S, rot, rho, R)


def test_tabu_replay_bounds_and_local_search_prefix():
    for seed in range(6):
        C, hel, rho = random_case(seed, B=11, M=35)
        K_r, K_f, R = 2, 2, 650
        if (1 - hel).sum() < K_f:
            continue
        S0, rot0 = oracle.fleet_rank(C, K_r, K_f, hel)
        tb = oracle.fleet_tabu(C, K_r, K_f, hel, rho, R, 3, 40)
        replay(C, hel, rho, R, S0, rot0, tb)
        opt = brute_np(C, K_r, K_f, hel, rho, R)
        assert (tb.coverage, -tb.distance) <= (opt[0], -opt[1])
        assert value_np(C, tb.best_open, tb.best_rot, rho, R) == (tb.coverage, tb.distance)
        ls = oracle.fleet_tabu(C, K_r, K_f, hel, rho, R, 3, 40, mode=1)
        n = int(ls.moved.sum())
        assert np.array_equal(ls.out_base[:n], tb.out_base[:n])
        assert np.array_equal(ls.in_base[:n], tb.in_base[:n])
        assert (ls.coverage, -ls.distance) <= (tb.coverage, -tb.distance)


def test_all_rotary_only_missions_ignore_fixed_wing():
    C, hel, _ = random_case(4, B=12, M=30)
    rho = np.ones(30, dtype=np.int32)
    S = np.array([0, 3, 5, 8])
    rot = np.array([1, 1, 0, 0], dtype=np.int32)
    assert oracle.fleet_value(C, S, rot, rho, 800) == oracle.placement_value(C, S[:2], 800)
