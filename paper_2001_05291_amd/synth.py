"""Seeded synthetic fleet-staging workloads.

The paper evaluates on random subsets of real aerodrome, heliport and hospital
coordinates in Ontario (Section 5); that data is not available here, so this
module draws synthetic stand-ins of the same structure: candidate bases
uniform over a lat/lon box, hospitals partly clustered around a few centres,
and missions as (pickup, delivery) hospital pairs (Section 3, mission tuple).

This module only produces inputs.  It holds none of the method's arithmetic
(no distance, no cost, no search), so both the CPU oracle's tests and the GPU
path can be fed from it without sharing any computation.

Random numbers come from a counter-based generator built on the SplitMix64
output function (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): draw ``k`` of stream ``s`` under ``seed`` is
``mix64(key(seed, s) + (k + 1) * GAMMA)`` with
``key(seed, s) = mix64(seed * GAMMA ^ s * 0xD1B54A32D192ED03)``, and a uniform
variate is ``(x >> 11) * 2**-53``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_STREAM_MUL = np.uint64(0xD1B54A32D192ED03)

# Bounding box of the synthetic region (degrees): lat 42..56 N, lon 95..74 W.
LAT0, LAT1 = 42.0, 56.0
LON0, LON1 = -95.0, -74.0
# Cluster centres lie in the southern band of the box, lat 42..46 N.
CLUSTER_LAT1 = 46.0
N_CLUSTERS = 5
CLUSTER_SIGMA_DEG = 1.0
CLUSTER_FRACTION = 0.7
MAX_REDRAWS = 64

# Stream ids (one per independent quantity).
_S_BASE_LAT, _S_BASE_LON = 1, 2
_S_CENTRE_LAT, _S_CENTRE_LON = 3, 4
_S_CLUSTER_OF = 5
_S_BM_U1, _S_BM_U2 = 6, 7
_S_HOSP_LAT, _S_HOSP_LON = 8, 9
_S_PICK, _S_DROP = 10, 11
_S_SIZES = 12
_S_PERTURB_PICK, _S_PERTURB_NEW = 13, 14
_S_ARRIVAL, _S_REQ_KIND, _S_REQ_PICK = 15, 16, 17
_S_POOL_RANGE = 18
_S_HELIPORT, _S_HOSP_ROTARY = 19, 20


def _mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * GAMMA
        s = s ^ (np.uint64(stream) * _STREAM_MUL)
    return _mix64(np.array([s], dtype=np.uint64))[0]


def raw(seed: int, stream: int, idx) -> np.ndarray:
    """Raw 64-bit draws number ``idx`` (array of non-negative ints) of a stream."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(_key(seed, stream) + (idx + np.uint64(1)) * GAMMA)


def uniform(seed: int, stream: int, idx) -> np.ndarray:
    """Uniform doubles in [0, 1) from draws ``idx`` of a stream."""
    return (raw(seed, stream, idx) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_int(seed: int, stream: int, idx, lo: int, hi: int) -> np.ndarray:
    """Integers uniform on {lo, ..., hi} (inclusive) via floor(lo + (hi-lo+1)*u)."""
    u = uniform(seed, stream, idx)
    return (lo + np.floor((hi - lo + 1) * u)).astype(np.int64)


@dataclass
class Instance:
    """One synthetic staging instance (coordinates in degrees)."""

    seed: int
    bases: np.ndarray          # (B, 2) float64: lat, lon
    hospitals: np.ndarray      # (H, 2) float64: lat, lon
    mission_ph: np.ndarray     # (M, 2) int32: pickup, delivery hospital ids
    missions: np.ndarray       # (M, 4) float64: plat, plon, dlat, dlon
    K: int = 0
    R: int = 0
    T: int = 0
    N: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def B(self) -> int:
        return int(self.bases.shape[0])

    @property
    def M(self) -> int:
        return int(self.missions.shape[0])


def gen_bases(seed: int, B: int) -> np.ndarray:
    i = np.arange(B)
    lat = LAT0 + (LAT1 - LAT0) * uniform(seed, _S_BASE_LAT, i)
    lon = LON0 + (LON1 - LON0) * uniform(seed, _S_BASE_LON, i)
    return np.ascontiguousarray(np.stack([lat, lon], axis=1))


def gen_hospitals(seed: int, H: int) -> np.ndarray:
    n_cl = int(np.floor(CLUSTER_FRACTION * H))
    c = np.arange(N_CLUSTERS)
    c_lat = LAT0 + (CLUSTER_LAT1 - LAT0) * uniform(seed, _S_CENTRE_LAT, c)
    c_lon = LON0 + (LON1 - LON0) * uniform(seed, _S_CENTRE_LON, c)
    h = np.arange(n_cl)
    which = np.minimum(np.floor(N_CLUSTERS * uniform(seed, _S_CLUSTER_OF, h)).astype(np.int64),
                       N_CLUSTERS - 1)
    lat = np.full(n_cl, np.nan)
    lon = np.full(n_cl, np.nan)
    pending = np.ones(n_cl, dtype=bool)
    for a in range(MAX_REDRAWS):
        if not pending.any():
            break
        hp = h[pending]
        draw = hp.astype(np.uint64) * np.uint64(MAX_REDRAWS) + np.uint64(a)
        u1 = 1.0 - uniform(seed, _S_BM_U1, draw)          # (0, 1]
        u2 = uniform(seed, _S_BM_U2, draw)
        rad = np.sqrt(-2.0 * np.log(u1))
        z0 = rad * np.cos(2.0 * np.pi * u2)
        z1 = rad * np.sin(2.0 * np.pi * u2)
        la = c_lat[which[hp]] + CLUSTER_SIGMA_DEG * z0
        lo = c_lon[which[hp]] + CLUSTER_SIGMA_DEG * z1
        ok = (la >= LAT0) & (la <= LAT1) & (lo >= LON0) & (lo <= LON1)
        idx = hp[ok]
        lat[idx] = la[ok]
        lon[idx] = lo[ok]
        pending[idx] = False
    if pending.any():  # practically unreachable; keep the draw inside the box
        hp = h[pending]
        lat[hp] = np.clip(c_lat[which[hp]], LAT0, LAT1)
        lon[hp] = np.clip(c_lon[which[hp]], LON0, LON1)
    u_idx = np.arange(H - n_cl)
    ulat = LAT0 + (LAT1 - LAT0) * uniform(seed, _S_HOSP_LAT, u_idx)
    ulon = LON0 + (LON1 - LON0) * uniform(seed, _S_HOSP_LON, u_idx)
    return np.ascontiguousarray(
        np.stack([np.concatenate([lat, ulat]), np.concatenate([lon, ulon])], axis=1))


def gen_mission_pairs(seed: int, H: int, M: int, first: int = 0,
                      streams=(_S_PICK, _S_DROP)) -> np.ndarray:
    """(M, 2) int32 distinct (pickup, delivery) hospital ids; p != d."""
    if H < 2:
        raise ValueError("need at least two hospitals for distinct pickup/delivery")
    k = np.arange(first, first + M)
    p = np.floor(H * uniform(seed, streams[0], k)).astype(np.int64)
    d = np.floor((H - 1) * uniform(seed, streams[1], k)).astype(np.int64)
    d = d + (d >= p)
    return np.ascontiguousarray(np.stack([p, d], axis=1).astype(np.int32))


def missions_from_pairs(hospitals: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    p = hospitals[pairs[:, 0]]
    d = hospitals[pairs[:, 1]]
    return np.ascontiguousarray(np.concatenate([p, d], axis=1))


def make_instance(seed: int, B: int, H: int, M: int, K: int = 0, R: int = 0,
                  T: int = 0, N: int = 0, **meta) -> Instance:
    bases = gen_bases(seed, B)
    hosp = gen_hospitals(seed, H)
    pairs = gen_mission_pairs(seed, H, M)
    return Instance(seed=seed, bases=bases, hospitals=hosp, mission_ph=pairs,
                    missions=missions_from_pairs(hosp, pairs), K=K, R=R, T=T, N=N,
                    meta=dict(meta))


# Single-instance workload presets (seed, sizes, range in metres, tenure, iterations).
WORKLOADS = {
    "small": dict(seed=0, B=40, H=120, M=200, K=5, R=1_200_000, T=7, N=100),
    "medium": dict(seed=0, B=500, H=1_500, M=20_000, K=30, R=1_000_000, T=15, N=500),
    "large": dict(seed=0, B=4_000, H=10_000, M=100_000, K=64, R=900_000, T=25, N=200),
}
# Heterogeneous fleet (Section 3 sets R and F, Eq. 10): a share of the
# candidate bases are heliports, a share of the hospitals can be reached by
# rotary-wing vehicles only (a mission touching one is rotary-only), and a
# share of the K vehicles are rotary-wing.
FLEET = dict(heliport_fraction=0.4, hospital_rotary_fraction=0.25, rotary_fraction=0.6)
BATCH = dict(n=1024, size_seed=4, T=10, N=200)
# Repositioning requests: 95% on instances shaped like the ragged batch, 5% on
# large ones; each redraws 10% of the missions and runs 100 iterations.
SERVE_LARGE = dict(B=2_000, H=6_000, M=50_000, K=48)
SERVE = dict(seed=5, large_fraction=0.05, redraw_fraction=0.1, T=10, N=100)


def workload_instance(name: str) -> Instance:
    c = dict(WORKLOADS[name])
    return make_instance(**c, workload=name)


def batch_sizes(n: int = 1024, size_seed: int = 4):
    """Per-instance (B, M, K, R) of the ragged batch: B~U{30..400}, M~U{100..5000},
    K~U{3..24}, R~U{800000..1400000} metres, H = 3B."""
    i = np.arange(n, dtype=np.int64)
    B = uniform_int(size_seed, _S_SIZES, 4 * i + 0, 30, 400)
    M = uniform_int(size_seed, _S_SIZES, 4 * i + 1, 100, 5000)
    K = uniform_int(size_seed, _S_SIZES, 4 * i + 2, 3, 24)
    R = uniform_int(size_seed, _S_SIZES, 4 * i + 3, 800_000, 1_400_000)
    return [dict(B=int(B[k]), H=3 * int(B[k]), M=int(M[k]), K=int(K[k]), R=int(R[k]))
            for k in range(n)]


def batch_instances(n: int = 1024, size_seed: int = 4, T: int = 10, N: int = 200):
    return [make_instance(seed=k, T=T, N=N, **s) for k, s in enumerate(batch_sizes(n, size_seed))]


def perturbation(seed: int, H: int, M: int, fraction: float = 0.1, request: int = 0):
    """A repositioning request: floor(fraction*M) distinct mission ids and a fresh
    distinct (pickup, delivery) hospital pair for each of them."""
    n = int(np.floor(fraction * M))
    # distinct ids by ranking M keyed draws (a seeded random permutation)
    keys = raw(seed, _S_PERTURB_PICK, np.arange(M, dtype=np.uint64) + np.uint64(M) * np.uint64(request))
    ids = np.sort(np.argsort(keys, kind="stable")[:n]).astype(np.int32)
    pairs = gen_mission_pairs(seed, H, n, first=request * M,
                              streams=(_S_PERTURB_NEW, _S_PERTURB_NEW + 100))
    return ids, pairs


def serve_pool(n_small: int, n_large: int, size_seed: int = 4):
    """Resident instances of the repositioning load: n_small shaped like the
    ragged batch (data seed = index) and n_large of SERVE_LARGE's size with a
    range drawn like the batch's (data seed = 100000 + index)."""
    pool = [make_instance(seed=k, **s) for k, s in enumerate(batch_sizes(n_small, size_seed))]
    rng = uniform_int(size_seed, _S_POOL_RANGE, np.arange(n_large), 800_000, 1_400_000)
    for k in range(n_large):
        pool.append(make_instance(seed=100_000 + k, R=int(rng[k]), **SERVE_LARGE))
    return pool


def request_stream(n: int, rate: float, n_small: int, n_large: int, seed: int = 5,
                   large_fraction: float = 0.05):
    """n requests of a Poisson arrival process of the given rate (per second;
    0 = all arrive at time 0): arrival times (s, ascending) and the pool index
    each request targets (a large instance with probability large_fraction,
    else a small one, uniformly within the kind)."""
    q = np.arange(n)
    if rate > 0:
        gaps = -np.log1p(-uniform(seed, _S_ARRIVAL, q)) / rate
        t = np.cumsum(gaps)
    else:
        t = np.zeros(n)
    large = (uniform(seed, _S_REQ_KIND, q) < large_fraction) & (n_large > 0)
    if n_small == 0:
        large[:] = True
    u = uniform(seed, _S_REQ_PICK, q)
    small_idx = np.minimum(np.floor(n_small * u).astype(np.int64), max(n_small - 1, 0))
    large_idx = n_small + np.minimum(np.floor(n_large * u).astype(np.int64), max(n_large - 1, 0))
    return t, np.where(large, large_idx, small_idx)


def fleet_flags(seed: int, B: int, mission_ph: np.ndarray, H: int,
                heliport_fraction: float = FLEET["heliport_fraction"],
                hospital_rotary_fraction: float = FLEET["hospital_rotary_fraction"]):
    """(heliport (B,) int32, rotary_only (M,) int32): base b is a heliport with
    probability heliport_fraction; a hospital is reachable by rotary-wing
    vehicles only with probability hospital_rotary_fraction, and a mission is
    rotary-only when its pickup or its delivery hospital is."""
    hel = (uniform(seed, _S_HELIPORT, np.arange(B)) < heliport_fraction).astype(np.int32)
    hosp = uniform(seed, _S_HOSP_ROTARY, np.arange(H)) < hospital_rotary_fraction
    ph = np.asarray(mission_ph)
    rho = (hosp[ph[:, 0]] | hosp[ph[:, 1]]).astype(np.int32)
    return hel, rho


def fleet_split(K: int, rotary_fraction: float = FLEET["rotary_fraction"]):
    """(K_r, K_f) with K_r = round(rotary_fraction * K)."""
    K_r = int(np.floor(rotary_fraction * K + 0.5))
    return K_r, K - K_r
