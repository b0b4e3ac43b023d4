"""CPU oracle for the fleet-staging hot path -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``liboracle.so`` (built from ``fleetstage_oracle.c``
by ``oracle/build.py``).  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
never does, and the two share no code.

Every function mirrors one routine of the C file, which cites the passage of
arXiv:2001.05291 it follows.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

EARTH_RADIUS_M = 6_371_000.0

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_c = ctypes
_lib = None


class _NullableArray:
    """ndpointer that also accepts None (passed as NULL)."""

    def __init__(self, base):
        self._base = base

    def from_param(self, obj):
        if obj is None:
            return None
        return self._base.from_param(obj)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, f64 = _c.c_int32, _c.c_int64, _c.c_double
    n_i32 = _NullableArray(_i32p)
    n_i64 = _NullableArray(_i64p)
    n_f64 = _NullableArray(_f64p)
    lib.fso_set_threads.argtypes = [_c.c_int]
    lib.fso_set_threads.restype = None
    lib.fso_get_threads.argtypes = []
    lib.fso_get_threads.restype = _c.c_int
    lib.fso_haversine.argtypes = [f64, f64, f64, f64, f64]
    lib.fso_haversine.restype = f64
    lib.fso_round_metres.argtypes = [f64]
    lib.fso_round_metres.restype = i32
    lib.fso_cost_table.argtypes = [_f64p, i32, _f64p, i32, f64, i32, n_f64, _i32p, i64]
    lib.fso_cost_table.restype = None
    lib.fso_row_sums.argtypes = [_i32p, i64, i32, i32, _i64p]
    lib.fso_row_sums.restype = None
    lib.fso_rank_bases.argtypes = [_i32p, i64, i32, i32, i32, _i32p, n_i32, n_i64]
    lib.fso_rank_bases.restype = None
    lib.fso_placement_value.argtypes = [_i32p, i64, i32, i32, _i32p, i32, i32,
                                        _c.POINTER(i32), _c.POINTER(i64)]
    lib.fso_placement_value.restype = None
    lib.fso_assign.argtypes = [_i32p, i64, i32, i32, _i32p, i32, i32, _i32p]
    lib.fso_assign.restype = None
    lib.fso_move_scores.argtypes = [_i32p, i64, i32, i32, _i32p, i32, i32, _i32p, _i64p]
    lib.fso_move_scores.restype = None
    lib.fso_tabu.argtypes = [_i32p, i64, i32, i32, i32, i32, i32, i32, i32, n_i32,
                             _i32p, _c.POINTER(i32), _c.POINTER(i64), _c.POINTER(i32),
                             n_i32, n_i32, n_i32, n_i32, n_i64, n_i32, n_i64]
    lib.fso_tabu.restype = _c.c_int
    lib.fso_brute_optimum.argtypes = [_i32p, i64, i32, i32, i32, i32, _i32p,
                                      _c.POINTER(i32), _c.POINTER(i64), _c.POINTER(i64)]
    lib.fso_brute_optimum.restype = None
    lib.fso_fleet_value.argtypes = [_i32p, i64, i32, _i32p, _i32p, i32, _i32p, i32,
                                    _c.POINTER(i32), _c.POINTER(i64)]
    lib.fso_fleet_value.restype = None
    lib.fso_fleet_assign.argtypes = [_i32p, i64, i32, _i32p, _i32p, i32, _i32p, i32, _i32p]
    lib.fso_fleet_assign.restype = None
    lib.fso_fleet_move_scores.argtypes = [_i32p, i64, i32, i32, _i32p, _i32p, i32, _i32p,
                                          _i32p, i32, _i32p, _i64p]
    lib.fso_fleet_move_scores.restype = None
    lib.fso_fleet_rank.argtypes = [_i32p, i64, i32, i32, i32, i32, _i32p, _i32p, _i32p]
    lib.fso_fleet_rank.restype = _c.c_int
    lib.fso_fleet_tabu.argtypes = [_i32p, i64, i32, i32, i32, i32, _i32p, _i32p, i32, i32, i32,
                                   i32, n_i32, n_i32, _i32p, _i32p, _c.POINTER(i32),
                                   _c.POINTER(i64), _c.POINTER(i32), n_i32, n_i32, n_i32, n_i32,
                                   n_i64, n_i32, n_i64]
    lib.fso_fleet_tabu.restype = _c.c_int
    lib.fso_fleet_brute_optimum.argtypes = [_i32p, i64, i32, i32, i32, i32, _i32p, _i32p, i32,
                                            _i32p, _i32p, _c.POINTER(i32), _c.POINTER(i64),
                                            _c.POINTER(i64)]
    lib.fso_fleet_brute_optimum.restype = None
    u64 = _c.c_uint64
    lib.fso_mix64.argtypes = [u64]
    lib.fso_mix64.restype = u64
    lib.fso_perm_priority.argtypes = [u64, i32, i32, i32, i32]
    lib.fso_perm_priority.restype = u64
    lib.fso_perm_search.argtypes = [_i32p, i64, i32, i32, i32, i32, i32, i32, i32, u64, n_i32,
                                    _i32p, _c.POINTER(i32), _c.POINTER(i64), _c.POINTER(i32),
                                    _c.POINTER(i32), n_i32, n_i32, n_i32, n_i32, n_i64, n_i32,
                                    n_i64]
    lib.fso_perm_search.restype = _c.c_int
    _lib = lib
    return lib


def set_threads(n: int) -> None:
    _load().fso_set_threads(int(n))


def get_threads() -> int:
    return int(_load().fso_get_threads())


def haversine(lat_a, lon_a, lat_b, lon_b, r: float = EARTH_RADIUS_M) -> float:
    return float(_load().fso_haversine(float(lat_a), float(lon_a), float(lat_b),
                                       float(lon_b), float(r)))


def round_metres(x: float) -> int:
    return int(_load().fso_round_metres(float(x)))


def cost_table(bases, missions, r: float = EARTH_RADIUS_M, legs: int = 3,
               want_cf: bool = True, ldc: int | None = None):
    """Returns (C int32 B x ldc, Cf float64 B x ldc or None)."""
    bases = np.ascontiguousarray(bases, dtype=np.float64)
    missions = np.ascontiguousarray(missions, dtype=np.float64)
    B, M = bases.shape[0], missions.shape[0]
    ldc = M if ldc is None else int(ldc)
    C = np.zeros((B, ldc), dtype=np.int32)
    Cf = np.zeros((B, ldc), dtype=np.float64) if want_cf else None
    _load().fso_cost_table(bases, B, missions, M, float(r), int(legs), Cf, C, ldc)
    return C, Cf


def _cm(C):
    C = np.ascontiguousarray(C, dtype=np.int32)
    return C, C.shape[0], C.shape[1]


def row_sums(C, M: int | None = None):
    C, B, ldc = _cm(C)
    M = ldc if M is None else M
    out = np.zeros(B, dtype=np.int64)
    _load().fso_row_sums(C, ldc, B, M, out)
    return out


def rank_bases(C, K: int, M: int | None = None):
    """Returns (open ascending, order chosen, row sums)."""
    C, B, ldc = _cm(C)
    M = ldc if M is None else M
    op = np.zeros(K, dtype=np.int32)
    order = np.zeros(K, dtype=np.int32)
    sums = np.zeros(B, dtype=np.int64)
    _load().fso_rank_bases(C, ldc, B, M, int(K), op, order, sums)
    return op, order, sums


def placement_value(C, S, R: int, M: int | None = None):
    C, B, ldc = _cm(C)
    M = ldc if M is None else M
    S = np.ascontiguousarray(S, dtype=np.int32)
    cov = _c.c_int32()
    dist = _c.c_int64()
    _load().fso_placement_value(C, ldc, B, M, S, S.shape[0], int(R), _c.byref(cov),
                                _c.byref(dist))
    return int(cov.value), int(dist.value)


def assign(C, S, R: int, M: int | None = None):
    C, B, ldc = _cm(C)
    M = ldc if M is None else M
    S = np.ascontiguousarray(S, dtype=np.int32)
    out = np.zeros(M, dtype=np.int32)
    _load().fso_assign(C, ldc, B, M, S, S.shape[0], int(R), out)
    return out


def move_scores(C, S, R: int, M: int | None = None):
    """(cov K x B, dist K x B); rows follow the slot order of S, closed columns only."""
    C, B, ldc = _cm(C)
    M = ldc if M is None else M
    S = np.ascontiguousarray(S, dtype=np.int32)
    K = S.shape[0]
    cov = np.zeros((K, B), dtype=np.int32)
    dist = np.zeros((K, B), dtype=np.int64)
    _load().fso_move_scores(C, ldc, B, M, S, K, int(R), cov, dist)
    return cov, dist


@dataclass
class TabuResult:
    best_open: np.ndarray
    coverage: int
    distance: int
    best_iter: int
    out_base: np.ndarray
    in_base: np.ndarray
    moved: np.ndarray
    cur_cov: np.ndarray
    cur_dist: np.ndarray
    best_cov: np.ndarray
    best_dist: np.ndarray


def tabu(C, K: int, R: int, T: int, N: int, mode: int = 0, init_open=None,
         M: int | None = None) -> TabuResult:
    C, B, ldc = _cm(C)
    M = ldc if M is None else M
    init = None if init_open is None else np.ascontiguousarray(init_open, dtype=np.int32)
    best = np.zeros(K, dtype=np.int32)
    cov = _c.c_int32()
    dist = _c.c_int64()
    it = _c.c_int32()
    n = max(int(N), 0)
    arr = [np.zeros(n, dtype=np.int32) for _ in range(4)]
    cur_d = np.zeros(n, dtype=np.int64)
    best_c = np.zeros(n, dtype=np.int32)
    best_d = np.zeros(n, dtype=np.int64)
    rc = _load().fso_tabu(C, ldc, B, M, int(K), int(R), int(T), int(N), int(mode), init, best,
                          _c.byref(cov), _c.byref(dist), _c.byref(it),
                          arr[0], arr[1], arr[2], arr[3], cur_d, best_c, best_d)
    if rc != 0:
        raise ValueError("oracle tabu: invalid arguments")
    return TabuResult(best, int(cov.value), int(dist.value), int(it.value), arr[0], arr[1],
                      arr[2], arr[3], cur_d, best_c, best_d)


def brute_optimum(C, K: int, R: int, M: int | None = None):
    C, B, ldc = _cm(C)
    M = ldc if M is None else M
    best = np.zeros(K, dtype=np.int32)
    cov = _c.c_int32()
    dist = _c.c_int64()
    n = _c.c_int64()
    _load().fso_brute_optimum(C, ldc, B, M, int(K), int(R), best, _c.byref(cov),
                              _c.byref(dist), _c.byref(n))
    return best, int(cov.value), int(dist.value), int(n.value)


# ---------------------------------------------------------------- heterogeneous fleet
# (Section 3, Eq. 2-10; readings in fleet_oracle.c)

def _flags(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(-1))
    if a.shape[0] != n:
        raise ValueError(f"expected {n} flags, got {a.shape[0]}")
    return a


def fleet_value(C, S, rot, rotary_only, R: int):
    C, B, M = _cm(C)
    S = np.ascontiguousarray(S, dtype=np.int32)
    rot = _flags(rot, S.shape[0])
    cov = _c.c_int32()
    dist = _c.c_int64()
    _load().fso_fleet_value(C, M, M, S, rot, S.shape[0], _flags(rotary_only, M), int(R),
                            _c.byref(cov), _c.byref(dist))
    return int(cov.value), int(dist.value)


def fleet_assign(C, S, rot, rotary_only, R: int):
    C, B, M = _cm(C)
    S = np.ascontiguousarray(S, dtype=np.int32)
    out = np.zeros(M, dtype=np.int32)
    _load().fso_fleet_assign(C, M, M, S, _flags(rot, S.shape[0]), S.shape[0],
                             _flags(rotary_only, M), int(R), out)
    return out


def fleet_move_scores(C, S, rot, heliport, rotary_only, R: int):
    """(cov K x B, dist K x B) of every relocation; -1 where not a move."""
    C, B, M = _cm(C)
    S = np.ascontiguousarray(S, dtype=np.int32)
    K = S.shape[0]
    cov = np.zeros((K, B), dtype=np.int32)
    dist = np.zeros((K, B), dtype=np.int64)
    _load().fso_fleet_move_scores(C, M, B, M, S, _flags(rot, K), K, _flags(heliport, B),
                                  _flags(rotary_only, M), int(R), cov, dist)
    return cov, dist


def fleet_rank(C, K_r: int, K_f: int, heliport):
    """(bases, rotary flags) in slot order; raises when the bases cannot hold the fleet."""
    C, B, M = _cm(C)
    K = int(K_r) + int(K_f)
    op = np.zeros(max(K, 1), dtype=np.int32)
    rot = np.zeros(max(K, 1), dtype=np.int32)
    if _load().fso_fleet_rank(C, M, B, M, int(K_r), int(K_f), _flags(heliport, B), op, rot):
        raise ValueError("the bases cannot hold the fleet")
    return op[:K], rot[:K]


@dataclass
class FleetResult(TabuResult):
    best_rot: np.ndarray = None   # rotary flags of best_open (ascending base ids)


def fleet_tabu(C, K_r: int, K_f: int, heliport, rotary_only, R: int, T: int, N: int,
               mode: int = 0, init_open=None, init_rot=None) -> FleetResult:
    """Typed Tabu search; the best placement is returned in ascending base-id
    order with the vehicle types permuted alongside."""
    C, B, M = _cm(C)
    K = int(K_r) + int(K_f)
    init = None if init_open is None else np.ascontiguousarray(init_open, dtype=np.int32)
    irot = None if init_rot is None else _flags(init_rot, K)
    best = np.zeros(K, dtype=np.int32)
    brot = np.zeros(K, dtype=np.int32)
    cov = _c.c_int32()
    dist = _c.c_int64()
    it = _c.c_int32()
    n = max(int(N), 0)
    arr = [np.zeros(n, dtype=np.int32) for _ in range(4)]
    cur_d = np.zeros(n, dtype=np.int64)
    best_c = np.zeros(n, dtype=np.int32)
    best_d = np.zeros(n, dtype=np.int64)
    rc = _load().fso_fleet_tabu(C, M, B, M, int(K_r), int(K_f), _flags(heliport, B),
                                _flags(rotary_only, M), int(R), int(T), int(N), int(mode),
                                init, irot, best, brot, _c.byref(cov), _c.byref(dist),
                                _c.byref(it), arr[0], arr[1], arr[2], arr[3], cur_d, best_c,
                                best_d)
    if rc != 0:
        raise ValueError("oracle fleet tabu: invalid arguments or bases cannot hold the fleet")
    order = np.argsort(best, kind="stable")
    return FleetResult(best[order], int(cov.value), int(dist.value), int(it.value), arr[0],
                       arr[1], arr[2], arr[3], cur_d, best_c, best_d, brot[order])


def fleet_brute_optimum(C, K_r: int, K_f: int, heliport, rotary_only, R: int):
    """(bases in slot order: rotary then fixed, types, cov, dist, placements)."""
    C, B, M = _cm(C)
    K = int(K_r) + int(K_f)
    best = np.zeros(max(K, 1), dtype=np.int32)
    brot = np.zeros(max(K, 1), dtype=np.int32)
    cov = _c.c_int32()
    dist = _c.c_int64()
    n = _c.c_int64()
    _load().fso_fleet_brute_optimum(C, M, B, M, int(K_r), int(K_f), _flags(heliport, B),
                                    _flags(rotary_only, M), int(R), best, brot, _c.byref(cov),
                                    _c.byref(dist), _c.byref(n))
    return best[:K], brot[:K], int(cov.value), int(dist.value), int(n.value)


# ---------------------------------------------------------------- permuted searches
# (Algorithms 2 and 3 with their random scan orders; readings in perm_oracle.c)

def mix64(z: int) -> int:
    """SplitMix64 output function."""
    return int(_load().fso_mix64(int(z) & (2**64 - 1)))


def perm_priority(seed: int, p: int, B: int, i: int, j: int) -> int:
    """Priority of swap (i out, j in) in pass p of a search seeded with seed."""
    return int(_load().fso_perm_priority(int(seed) & (2**64 - 1), int(p), int(B), int(i), int(j)))


@dataclass
class PermResult(TabuResult):
    passes: int = 0


def perm_search(C, K: int, R: int, T: int, N: int, mode: int, seed: int, init_open=None,
                M: int | None = None) -> PermResult:
    """Permuted first-improvement search: mode 2 local search, mode 3 Tabu
    with improving-only acceptance."""
    C, B, ldc = _cm(C)
    M = ldc if M is None else M
    init = None if init_open is None else np.ascontiguousarray(init_open, dtype=np.int32)
    best = np.zeros(K, dtype=np.int32)
    cov = _c.c_int32()
    dist = _c.c_int64()
    it = _c.c_int32()
    passes = _c.c_int32()
    n = max(int(N), 0)
    arr = [np.zeros(n, dtype=np.int32) for _ in range(4)]
    cur_d = np.zeros(n, dtype=np.int64)
    best_c = np.zeros(n, dtype=np.int32)
    best_d = np.zeros(n, dtype=np.int64)
    rc = _load().fso_perm_search(C, ldc, B, M, int(K), int(R), int(T), int(N), int(mode),
                                 int(seed) & (2**64 - 1), init, best, _c.byref(cov),
                                 _c.byref(dist), _c.byref(it), _c.byref(passes), arr[0], arr[1],
                                 arr[2], arr[3], cur_d, best_c, best_d)
    if rc != 0:
        raise ValueError("oracle permuted search: invalid arguments")
    return PermResult(best, int(cov.value), int(dist.value), int(it.value), arr[0], arr[1],
                      arr[2], arr[3], cur_d, best_c, best_d, int(passes.value))
