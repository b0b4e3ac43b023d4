"""Pins of the oracle's distance model (Eq. 1) and cost table (Algorithm 1's
Distances fill) against closed forms and an independent great-circle formula.
CPU only."""

import math

import numpy as np
import pytest

import oracle
from paper_2001_05291_amd import synth

R_EARTH = 6_371_000.0


def vincenty_sphere(lat1, lon1, lat2, lon2, r=R_EARTH):
    """Great-circle distance by the atan2 (Vincenty, sphere) form: a formula
    different from the haversine of Eq. 1 but equal to it in exact arithmetic."""
    p1, p2 = np.radians(lat1), np.radians(lat2)
    dl = np.radians(lon2) - np.radians(lon1)
    num = np.hypot(np.cos(p2) * np.sin(dl),
                   np.cos(p1) * np.sin(p2) - np.sin(p1) * np.cos(p2) * np.cos(dl))
    den = np.sin(p1) * np.sin(p2) + np.cos(p1) * np.cos(p2) * np.cos(dl)
    return r * np.arctan2(num, den)


def test_same_point_is_zero_exactly():
    for lat, lon in [(0, 0), (45.5, -80.25), (-89.9, 179.9), (56, -95)]:
        assert oracle.haversine(lat, lon, lat, lon) == 0.0


def test_one_degree_of_latitude():
    # r * pi / 180 with r = 6,371,000 m
    assert abs(oracle.haversine(44.0, -80.0, 45.0, -80.0) - 111194.92664455874) < 1e-6


@pytest.mark.parametrize("lat1,lat2", [(0.0, 10.0), (42.0, 56.0), (-30.0, 60.0), (50.0, 50.001)])
def test_meridian_arc(lat1, lat2):
    d = oracle.haversine(lat1, -85.0, lat2, -85.0)
    exact = R_EARTH * abs(math.radians(lat2) - math.radians(lat1))
    assert d == pytest.approx(exact, rel=1e-13)


@pytest.mark.parametrize("lon1,lon2", [(0.0, 1.0), (-95.0, -74.0), (-170.0, 10.0), (3.0, 3.0001)])
def test_equator_arc(lon1, lon2):
    d = oracle.haversine(0.0, lon1, 0.0, lon2)
    exact = R_EARTH * abs(math.radians(lon2) - math.radians(lon1))
    assert d == pytest.approx(exact, rel=1e-13)


def test_antipodes_and_clamp():
    assert oracle.haversine(0.0, 0.0, 0.0, 180.0) == pytest.approx(math.pi * R_EARTH, rel=1e-15)
    # poles: the radicand rounds above 1 and must be clamped, not NaN
    d = oracle.haversine(90.0, 0.0, -90.0, 0.0)
    assert d == pytest.approx(math.pi * R_EARTH, rel=1e-15)


def test_radius_scales_linearly():
    a = oracle.haversine(43.0, -79.0, 48.4, -89.2, r=1.0)
    b = oracle.haversine(43.0, -79.0, 48.4, -89.2, r=R_EARTH)
    assert b == pytest.approx(a * R_EARTH, rel=1e-15)


def test_haversine_matches_independent_formula():
    rng = np.random.default_rng(1)
    n = 2000
    lat1 = rng.uniform(-80, 80, n)
    lon1 = rng.uniform(-180, 180, n)
    # mixture of near and far pairs
    scale = np.where(rng.random(n) < 0.5, 1e-3, 40.0)
    lat2 = np.clip(lat1 + scale * rng.normal(size=n), -89, 89)
    lon2 = lon1 + scale * rng.normal(size=n)
    ref = vincenty_sphere(lat1, lon1, lat2, lon2)
    got = np.array([oracle.haversine(*a) for a in zip(lat1, lon1, lat2, lon2)])
    assert np.all(np.abs(got - ref) <= 1e-12 * ref + 1e-9)


def test_round_half_even():
    assert oracle.round_metres(2.5) == 2
    assert oracle.round_metres(3.5) == 4
    assert oracle.round_metres(10_000_000.5) == 10_000_000
    assert oracle.round_metres(10_000_001.5) == 10_000_002
    assert oracle.round_metres(7.4999999) == 7
    assert oracle.round_metres(7.5000001) == 8


def _legs(inst):
    b = inst.bases
    ms = inst.missions
    bp = vincenty_sphere(b[:, None, 0], b[:, None, 1], ms[None, :, 0], ms[None, :, 1])
    pd = vincenty_sphere(ms[:, 0], ms[:, 1], ms[:, 2], ms[:, 3])[None, :]
    db = vincenty_sphere(ms[None, :, 2], ms[None, :, 3], b[:, None, 0], b[:, None, 1])
    return bp, pd, db


def test_cost_table_three_legs_matches_independent_sum():
    inst = synth.make_instance(seed=7, B=30, H=60, M=50)
    C, Cf = oracle.cost_table(inst.bases, inst.missions, legs=3)
    bp, pd, db = _legs(inst)
    ref = bp + pd + db
    assert np.all(np.abs(Cf - ref) <= 1e-12 * ref)
    # int32 metres, rounded half to even from the float table
    assert C.dtype == np.int32
    assert np.array_equal(C, np.rint(Cf).astype(np.int32))
    # round trip: at least the out-and-back between pickup and delivery
    assert np.all(Cf >= 2.0 * pd * (1 - 1e-12))


def test_cost_table_two_legs_drops_pickup_delivery():
    inst = synth.make_instance(seed=8, B=20, H=40, M=40)
    _, Cf3 = oracle.cost_table(inst.bases, inst.missions, legs=3)
    _, Cf2 = oracle.cost_table(inst.bases, inst.missions, legs=2)
    bp, pd, db = _legs(inst)
    assert np.all(np.abs(Cf2 - (bp + db)) <= 1e-12 * (bp + db))
    assert np.all(np.abs((Cf3 - Cf2) - pd) <= 1e-12 * Cf3)


def test_cost_table_reverse_mission_symmetry():
    inst = synth.make_instance(seed=9, B=16, H=30, M=25)
    rev = inst.missions[:, [2, 3, 0, 1]]
    _, Cf = oracle.cost_table(inst.bases, inst.missions)
    _, Cr = oracle.cost_table(inst.bases, rev)
    assert np.all(np.abs(Cf - Cr) <= 1e-12 * Cf)


def test_cost_table_row_pitch():
    inst = synth.make_instance(seed=10, B=9, H=20, M=13)
    C, Cf = oracle.cost_table(inst.bases, inst.missions)
    Cp, Cfp = oracle.cost_table(inst.bases, inst.missions, ldc=16)
    assert np.array_equal(Cp[:, :13], C)
    assert np.array_equal(Cfp[:, :13], Cf)


def test_cost_table_thread_count_invariant():
    inst = synth.make_instance(seed=11, B=40, H=50, M=60)
    n = oracle.get_threads()
    oracle.set_threads(1)
    C1, Cf1 = oracle.cost_table(inst.bases, inst.missions)
    oracle.set_threads(max(n, 2))
    C2, Cf2 = oracle.cost_table(inst.bases, inst.missions)
    oracle.set_threads(n)
    assert np.array_equal(C1, C2) and np.array_equal(Cf1, Cf2)
