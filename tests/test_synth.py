"""The synthetic input generators: determinism, shapes and the stated
distributions (CPU only; no method arithmetic is involved)."""

import numpy as np

from paper_2001_05291_amd import synth


def test_instance_is_deterministic_and_in_the_box():
    a = synth.make_instance(seed=3, B=50, H=90, M=400)
    b = synth.make_instance(seed=3, B=50, H=90, M=400)
    assert np.array_equal(a.missions, b.missions) and np.array_equal(a.bases, b.bases)
    for xy in (a.bases, a.hospitals):
        assert np.all((xy[:, 0] >= synth.LAT0) & (xy[:, 0] <= synth.LAT1))
        assert np.all((xy[:, 1] >= synth.LON0) & (xy[:, 1] <= synth.LON1))
    assert np.all(a.mission_ph[:, 0] != a.mission_ph[:, 1])


def test_batch_sizes_within_stated_ranges():
    sizes = synth.batch_sizes(1024)
    B = np.array([s["B"] for s in sizes])
    M = np.array([s["M"] for s in sizes])
    K = np.array([s["K"] for s in sizes])
    R = np.array([s["R"] for s in sizes])
    assert B.min() >= 30 and B.max() <= 400
    assert M.min() >= 100 and M.max() <= 5000
    assert K.min() >= 3 and K.max() <= 24
    assert R.min() >= 800_000 and R.max() <= 1_400_000
    assert all(s["H"] == 3 * s["B"] for s in sizes)


def test_perturbation_ids_distinct_and_sorted():
    ids, pairs = synth.perturbation(5, 300, 2000, 0.1, request=7)
    assert ids.size == 200 and np.all(np.diff(ids) > 0)
    assert ids.min() >= 0 and ids.max() < 2000
    assert np.all(pairs[:, 0] != pairs[:, 1])
    ids2, _ = synth.perturbation(5, 300, 2000, 0.1, request=8)
    assert not np.array_equal(ids, ids2)


def test_request_stream_poisson_rate_and_mix():
    n, rate = 20000, 250.0
    t, idx = synth.request_stream(n, rate, 1024, 64, seed=5)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps >= 0)
    # exponential gaps: mean 1/rate and coefficient of variation 1
    assert abs(gaps.mean() * rate - 1) < 0.03
    assert abs(gaps.std() / gaps.mean() - 1) < 0.03
    large = idx >= 1024
    assert abs(large.mean() - 0.05) < 0.01
    assert idx.min() >= 0 and idx.max() < 1024 + 64
    # the targets do not depend on the rate
    _, idx0 = synth.request_stream(n, 0.0, 1024, 64, seed=5)
    assert np.array_equal(idx, idx0)


def test_serve_pool_shapes():
    pool = synth.serve_pool(4, 2)
    assert len(pool) == 6
    assert all(w.B == synth.SERVE_LARGE["B"] and w.M == synth.SERVE_LARGE["M"]
               and w.K == synth.SERVE_LARGE["K"] for w in pool[4:])
    assert all(800_000 <= w.R <= 1_400_000 for w in pool)


def test_fleet_flags_deterministic_and_consistent():
    inst = synth.make_instance(seed=7, B=300, H=400, M=3000)
    hel, rho = synth.fleet_flags(7, inst.B, inst.mission_ph, 400)
    hel2, rho2 = synth.fleet_flags(7, inst.B, inst.mission_ph, 400)
    assert np.array_equal(hel, hel2) and np.array_equal(rho, rho2)
    assert hel.shape == (300,) and rho.shape == (3000,)
    assert set(np.unique(hel)) <= {0, 1} and set(np.unique(rho)) <= {0, 1}
    assert 0.3 < hel.mean() < 0.5
    # P(rotary-only) = 1 - (1 - 0.25)^2 for distinct endpoints
    assert 0.36 < rho.mean() < 0.51
    # a hospital on a mission that either type may fly is not rotary-only, so
    # a rotary-only mission has at least one endpoint outside that set
    ph = inst.mission_ph
    clear = np.zeros(400, dtype=bool)
    clear[ph[rho == 0].reshape(-1)] = True
    assert not np.any(clear[ph[rho == 1, 0]] & clear[ph[rho == 1, 1]])
    assert synth.fleet_split(30) == (18, 12) and synth.fleet_split(5) == (3, 2)
