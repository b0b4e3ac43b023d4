"""ctypes binding of libfleetstage.so (declared in include/fleetstage.h).

Argument marshalling only: every step runs in the HIP library.  PyTorch
provides device memory (CUDA/HIP tensors) and the current stream.  The binding
fails loudly when the library has not been built; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfleetstage.so")

FS_OK, FS_PENDING = 0, 1
FS_E_INVALID, FS_E_NOMEM, FS_E_DEVICE = -1, -2, -3
FS_E_BUDGET, FS_E_NOTFOUND, FS_E_CLOSED, FS_E_INTERNAL = -4, -5, -6, -7

TRACE_DTYPE = np.dtype([("iter", "<i4"), ("out_base", "<i4"), ("in_base", "<i4"),
                        ("moved", "<i4"), ("cur_cov", "<i4"), ("best_cov", "<i4"),
                        ("cur_dist", "<i8"), ("best_dist", "<i8")])
assert TRACE_DTYPE.itemsize == 40


class FleetstageError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"fleetstage status {status}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("tenure", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("range_m", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


assert ctypes.sizeof(Params) == 24

# search modes: Tabu (best admissible move, aspiration), steepest local search,
# and the paper's permuted local search / permuted Tabu search
MODE_TABU, MODE_LOCAL, MODE_PERM_LOCAL, MODE_PERM_TABU = 0, 1, 2, 3


class Score(ctypes.Structure):
    _fields_ = [("coverage", ctypes.c_int32), ("best_iter", ctypes.c_int32),
                ("distance", ctypes.c_int64)]


class Instance(ctypes.Structure):
    _fields_ = [("C", ctypes.c_void_p), ("ldc", ctypes.c_int64), ("B", ctypes.c_int32),
                ("M", ctypes.c_int32), ("K", ctypes.c_int32), ("range_m", ctypes.c_int32),
                ("init_open", ctypes.c_void_p), ("best_open_out", ctypes.c_void_p),
                ("assign_out", ctypes.c_void_p), ("trace_out", ctypes.c_void_p),
                ("seed", ctypes.c_uint64)]


assert ctypes.sizeof(Instance) == 72


class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("device", ctypes.c_int32), ("earth_radius_m", ctypes.c_double),
                ("legs", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ServeStats(ctypes.Structure):
    _fields_ = [("resident_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("evictions", ctypes.c_int64), ("rebuilds", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("running", ctypes.c_int32), ("queued", ctypes.c_int32)]


class Fleet(ctypes.Structure):
    _fields_ = [("rotary", ctypes.c_int32), ("fixed", ctypes.c_int32),
                ("heliport", ctypes.c_void_p), ("rotary_only", ctypes.c_void_p)]

_lib = None


def lib():
    """The loaded library (loads it on first use; raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FleetstageError(FS_E_DEVICE, f"{LIB_PATH} is not built; run "
                              "`python -m paper_2001_05291_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.fs_last_error.restype = ctypes.c_char_p
    L.fs_last_error.argtypes = []
    L.fs_version.restype = ctypes.c_char_p
    L.fs_version.argtypes = []
    L.fs_build_cost_table.restype = i32
    L.fs_build_cost_table.argtypes = [vp, i32, vp, i32, f64, i32, vp, i64, vp, vp]
    L.fs_build_cost_table_indexed.restype = i32
    L.fs_build_cost_table_indexed.argtypes = [vp, i32, vp, i32, vp, i32, f64, i32, vp, i64, vp,
                                              vp]
    L.fs_rank_bases.restype = i32
    L.fs_rank_bases.argtypes = [vp, i64, i32, i32, i32, vp, vp, vp, vp]
    L.fs_move_scores.restype = i32
    L.fs_move_scores.argtypes = [vp, i64, i32, i32, vp, i32, i32, vp, vp, vp]
    L.fs_tabu_solve.restype = i32
    L.fs_tabu_solve.argtypes = [vp, i64, i32, i32, i32, ctypes.POINTER(Params), vp, vp,
                                ctypes.POINTER(Score), vp, vp, vp]
    L.fs_tabu_solve_noalloc.restype = i32
    L.fs_tabu_solve_noalloc.argtypes = L.fs_tabu_solve.argtypes
    L.fs_noalloc_scratch_bytes.restype = i64
    L.fs_noalloc_scratch_bytes.argtypes = []
    L.fs_brute_optimum.restype = i32
    L.fs_brute_optimum.argtypes = [vp, i64, i32, i32, i32, i32, vp, ctypes.POINTER(Score),
                                   ctypes.POINTER(i64), vp]
    L.fs_fleet_move_scores.restype = i32
    L.fs_fleet_move_scores.argtypes = [vp, i64, i32, i32, ctypes.POINTER(Fleet), vp, vp, i32,
                                       vp, vp, vp]
    L.fs_fleet_solve.restype = i32
    L.fs_fleet_solve.argtypes = [vp, i64, i32, i32, ctypes.POINTER(Fleet),
                                 ctypes.POINTER(Params), vp, vp, vp, vp, ctypes.POINTER(Score),
                                 vp, vp, vp]
    L.fs_tabu_solve_batch.restype = i32
    L.fs_tabu_solve_batch.argtypes = [ctypes.POINTER(Instance), i32, ctypes.POINTER(Params),
                                      ctypes.POINTER(Score), vp]
    L.fs_serve_open.restype = i32
    L.fs_serve_open.argtypes = [ctypes.POINTER(ServeConfig), ctypes.POINTER(vp)]
    L.fs_serve_register.restype = i32
    L.fs_serve_register.argtypes = [vp, vp, i32, vp, i32, i32, i32, ctypes.POINTER(i64)]
    L.fs_serve_submit.restype = i32
    L.fs_serve_submit.argtypes = [vp, i64, vp, vp, i32, ctypes.POINTER(Params),
                                  ctypes.POINTER(ctypes.c_uint64)]
    L.fs_serve_poll.restype = i32
    L.fs_serve_poll.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(Score),
                                ctypes.POINTER(f64)]
    L.fs_serve_stats_get.restype = i32
    L.fs_serve_stats_get.argtypes = [vp, ctypes.POINTER(ServeStats)]
    L.fs_serve_close.restype = i32
    L.fs_serve_close.argtypes = [vp]
    L.fs_timing_enable.restype = i32
    L.fs_timing_enable.argtypes = [i32]
    L.fs_timing_read.restype = i32
    L.fs_timing_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(f64), ctypes.POINTER(i64)]
    _lib = L
    return L


def _check(status: int):
    if status != FS_OK:
        raise FleetstageError(status, lib().fs_last_error().decode(errors="replace"))


def _ptr(t, dtype=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device (cuda/hip) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _table(C, M):
    """(B, M, ldc) of a cost table: a (B, M) tensor whose rows are contiguous
    and ldc elements apart (what build_cost_table returns: a view of a B x ldc
    buffer), or a B x ldc buffer with the mission count M given explicitly."""
    if not isinstance(C, torch.Tensor) or C.dim() != 2 or C.dtype != torch.int32:
        raise TypeError("cost table must be a 2-D int32 tensor (bases x missions)")
    if not C.is_cuda:
        raise TypeError("expected a device (cuda/hip) tensor")
    B, width = C.shape
    if C.stride(1) != 1 and width > 1:
        raise ValueError("cost table rows must be contiguous")
    ldc = C.stride(0)
    if ldc < width:
        raise ValueError("cost table row stride is smaller than its width")
    M = width if M is None else int(M)
    if M > width:
        raise ValueError(f"M={M} exceeds the table width {width}")
    return B, M, ldc


def _table_ptr(C):
    return ctypes.c_void_p(C.data_ptr())


def version() -> str:
    return lib().fs_version().decode()


def build_cost_table(bases, missions, earth_radius_m: float = 0.0, legs: int = 3,
                     ldc: int | None = None, want_cf: bool = False, stream=None):
    """C (int32) and optionally Cf (float64) from device coordinates: bases
    (B, 2) and missions (M, 4) float64 degrees.  Both are (B, M) views of
    buffers with row pitch ldc, which defaults to M rounded up to a multiple
    of 4 (16-byte aligned rows)."""
    B, M = int(bases.shape[0]), int(missions.shape[0])
    ldc = (M + 3) // 4 * 4 if ldc is None else int(ldc)
    dev = bases.device
    C = torch.empty((B, ldc), dtype=torch.int32, device=dev)
    Cf = torch.empty((B, ldc), dtype=torch.float64, device=dev) if want_cf else None
    _check(lib().fs_build_cost_table(_ptr(bases, torch.float64), B,
                                     _ptr(missions, torch.float64), M, float(earth_radius_m),
                                     int(legs), _ptr(C), ldc, _ptr(Cf), _stream(stream)))
    # (B, M) views of the padded rows: the other calls read M and ldc from them
    return C[:, :M], (Cf[:, :M] if Cf is not None else None)


def build_cost_table_indexed(bases, hospitals, mission_ph, earth_radius_m: float = 0.0,
                             legs: int = 3, ldc: int | None = None, want_cf: bool = False,
                             stream=None):
    """As build_cost_table, from hospital coordinates (H, 2) float64 and the
    missions' (pickup, delivery) hospital ids (M, 2) int32, all on the
    device; bitwise the direct form's table."""
    B, H, M = int(bases.shape[0]), int(hospitals.shape[0]), int(mission_ph.shape[0])
    ldc = (M + 3) // 4 * 4 if ldc is None else int(ldc)
    dev = bases.device
    C = torch.empty((B, ldc), dtype=torch.int32, device=dev)
    Cf = torch.empty((B, ldc), dtype=torch.float64, device=dev) if want_cf else None
    _check(lib().fs_build_cost_table_indexed(_ptr(bases, torch.float64), B,
                                             _ptr(hospitals, torch.float64), H,
                                             _ptr(mission_ph, torch.int32), M,
                                             float(earth_radius_m), int(legs), _ptr(C), ldc,
                                             _ptr(Cf), _stream(stream)))
    return C[:, :M], (Cf[:, :M] if Cf is not None else None)


def rank_bases(C, K: int, M: int | None = None, stream=None):
    """(open ascending, order by rank, row sums) as device tensors."""
    B, M, ldc = _table(C, M)
    dev = C.device
    op = torch.empty(K, dtype=torch.int32, device=dev)
    order = torch.empty(K, dtype=torch.int32, device=dev)
    sums = torch.empty(B, dtype=torch.int64, device=dev)
    _check(lib().fs_rank_bases(_table_ptr(C), ldc, B, M, int(K), _ptr(op), _ptr(order), _ptr(sums),
                               _stream(stream)))
    return op, order, sums


def move_scores(C, open_ids, range_m: int, M: int | None = None, stream=None):
    """(cov, dist) device tensors K x B: value of open - open[k] + j for closed j."""
    B, M, ldc = _table(C, M)
    dev = C.device
    op = open_ids.to(device=dev, dtype=torch.int32).contiguous()
    K = int(op.numel())
    cov = torch.empty((K, B), dtype=torch.int32, device=dev)
    dist = torch.empty((K, B), dtype=torch.int64, device=dev)
    _check(lib().fs_move_scores(_table_ptr(C), ldc, B, M, _ptr(op), K, int(range_m), _ptr(cov),
                                _ptr(dist), _stream(stream)))
    return cov, dist


@dataclass
class SolveResult:
    best_open: torch.Tensor          # device int32 K, ascending
    coverage: int
    distance: int
    best_iter: int
    assign: torch.Tensor | None      # device int32 M
    trace: np.ndarray | None         # host structured array (TRACE_DTYPE)


def _tabu_solve(entry, C, K, range_m, tenure, iterations, mode, init_open, M, want_assign,
                want_trace, stream, seed):
    B, M, ldc = _table(C, M)
    dev = C.device
    p = Params(int(tenure), int(iterations), int(range_m), int(mode), int(seed) % 2**64)
    best = torch.empty(K, dtype=torch.int32, device=dev)
    assign = torch.empty(M, dtype=torch.int32, device=dev) if want_assign else None
    n = max(int(iterations), 0)
    trace = torch.empty(max(n, 1) * TRACE_DTYPE.itemsize, dtype=torch.uint8, device=dev) \
        if want_trace else None
    init = None
    if init_open is not None:
        init = init_open.to(device=dev, dtype=torch.int32).contiguous()
    sc = Score()
    _check(entry(_table_ptr(C), ldc, B, M, int(K), ctypes.byref(p), _ptr(init),
                 _ptr(best), ctypes.byref(sc), _ptr(assign),
                 _ptr(trace) if n > 0 else None, _stream(stream)))
    tr = None
    if want_trace:
        tr = trace[: n * TRACE_DTYPE.itemsize].cpu().numpy().view(TRACE_DTYPE)
    return SolveResult(best, int(sc.coverage), int(sc.distance), int(sc.best_iter), assign, tr)


def tabu_solve(C, K: int, range_m: int, tenure: int, iterations: int, mode: int = 0,
               init_open=None, M: int | None = None, want_assign: bool = True,
               want_trace: bool = True, stream=None, seed: int = 0) -> SolveResult:
    return _tabu_solve(lib().fs_tabu_solve, C, K, range_m, tenure, iterations, mode, init_open,
                       M, want_assign, want_trace, stream, seed)


def tabu_solve_noalloc(C, K: int, range_m: int, tenure: int, iterations: int, mode: int = 0,
                       init_open=None, M: int | None = None, want_assign: bool = True,
                       want_trace: bool = True, stream=None, seed: int = 0) -> SolveResult:
    """fs_tabu_solve_noalloc: the solve in the library's static device
    workspace (the output tensors are allocated here, by the caller side)."""
    return _tabu_solve(lib().fs_tabu_solve_noalloc, C, K, range_m, tenure, iterations, mode,
                       init_open, M, want_assign, want_trace, stream, seed)


def noalloc_scratch_bytes() -> int:
    return int(lib().fs_noalloc_scratch_bytes())


def tabu_solve_batch(instances, tenure: int, iterations: int, mode: int = 0,
                     want_assign: bool = True, want_trace: bool = True, stream=None):
    """Solves many instances in one launch set.  Each item is a dict with keys
    C (device int32 table), K, range_m, and optionally M, init_open and seed
    (scan orders of modes 2 and 3).  Returns one SolveResult per instance
    (identical to tabu_solve alone)."""
    n = len(instances)
    arr = (Instance * n)()
    keep = []
    outs = []
    nrec = max(int(iterations), 0)
    for i, it in enumerate(instances):
        C = it["C"]
        B, M, ldc = _table(C, it.get("M"))
        K = int(it["K"])
        dev = C.device
        best = torch.empty(K, dtype=torch.int32, device=dev)
        assign = torch.empty(M, dtype=torch.int32, device=dev) if want_assign else None
        trace = torch.empty(max(nrec, 1) * TRACE_DTYPE.itemsize, dtype=torch.uint8, device=dev) \
            if want_trace else None
        init = it.get("init_open")
        if init is not None:
            init = init.to(device=dev, dtype=torch.int32).contiguous()
        keep += [C, init]
        outs.append((best, assign, trace))
        arr[i].C = C.data_ptr()
        arr[i].ldc = ldc
        arr[i].B, arr[i].M, arr[i].K = B, M, K
        arr[i].range_m = int(it["range_m"])
        arr[i].init_open = init.data_ptr() if init is not None else None
        arr[i].best_open_out = best.data_ptr()
        arr[i].assign_out = assign.data_ptr() if assign is not None else None
        arr[i].trace_out = trace.data_ptr() if (trace is not None and nrec > 0) else None
        arr[i].seed = int(it.get("seed", 0)) % 2**64
    p = Params(int(tenure), int(iterations), 0, int(mode))
    scores = (Score * n)()
    _check(lib().fs_tabu_solve_batch(arr, n, ctypes.byref(p), scores, _stream(stream)))
    res = []
    for i, (best, assign, trace) in enumerate(outs):
        tr = None
        if trace is not None:
            tr = trace[: nrec * TRACE_DTYPE.itemsize].cpu().numpy().view(TRACE_DTYPE)
        res.append(SolveResult(best, int(scores[i].coverage), int(scores[i].distance),
                               int(scores[i].best_iter), assign, tr))
    return res


def brute_optimum(C, K: int, range_m: int, M: int | None = None, stream=None):
    """Exact optimum by enumeration of all K-subsets (small instances):
    (best_open device int32 K ascending, coverage, distance, placements)."""
    B, M, ldc = _table(C, M)
    best = torch.empty(int(K), dtype=torch.int32, device=C.device)
    sc = Score()
    n = ctypes.c_int64()
    _check(lib().fs_brute_optimum(_table_ptr(C), ldc, B, M, int(K), int(range_m), _ptr(best),
                                  ctypes.byref(sc), ctypes.byref(n), _stream(stream)))
    return best, int(sc.coverage), int(sc.distance), int(n.value)


# ---------------------------------------------------------------- heterogeneous fleet


def _fleet(K_r, K_f, heliport, rotary_only, dev, B, M):
    hel = torch.as_tensor(heliport).to(device=dev, dtype=torch.int32).contiguous()
    if hel.numel() != B:
        raise ValueError(f"heliport flags: expected {B}, got {hel.numel()}")
    rho = None
    if rotary_only is not None:
        rho = torch.as_tensor(rotary_only).to(device=dev, dtype=torch.int32).contiguous()
        if rho.numel() != M:
            raise ValueError(f"rotary-only flags: expected {M}, got {rho.numel()}")
    f = Fleet(int(K_r), int(K_f), hel.data_ptr(), rho.data_ptr() if rho is not None else None)
    return f, (hel, rho)


def fleet_move_scores(C, K_r: int, K_f: int, heliport, rotary_only, open_ids, rotary,
                      range_m: int, M: int | None = None, stream=None):
    """(cov, dist) device tensors K x B: value of the placement with the vehicle
    of slot k moved to base j; -1 where j is occupied or a heliport the vehicle
    cannot use."""
    B, M, ldc = _table(C, M)
    dev = C.device
    f, keep = _fleet(K_r, K_f, heliport, rotary_only, dev, B, M)
    op = torch.as_tensor(open_ids).to(device=dev, dtype=torch.int32).contiguous()
    rt = torch.as_tensor(rotary).to(device=dev, dtype=torch.int32).contiguous()
    K = int(K_r) + int(K_f)
    if op.numel() != K or rt.numel() != K:
        raise ValueError(f"placement and types must hold K={K} entries")
    cov = torch.empty((K, B), dtype=torch.int32, device=dev)
    dist = torch.empty((K, B), dtype=torch.int64, device=dev)
    _check(lib().fs_fleet_move_scores(_table_ptr(C), ldc, B, M, ctypes.byref(f), _ptr(op),
                                      _ptr(rt), int(range_m), _ptr(cov), _ptr(dist),
                                      _stream(stream)))
    return cov, dist


@dataclass
class FleetResult(SolveResult):
    best_rotary: torch.Tensor = None   # device int32 K: types of best_open (1 = rotary-wing)


def fleet_solve(C, K_r: int, K_f: int, heliport, rotary_only, range_m: int, tenure: int,
                iterations: int, mode: int = 0, init_open=None, init_rotary=None,
                M: int | None = None, want_assign: bool = True, want_trace: bool = True,
                stream=None, seed: int = 0) -> FleetResult:
    """Typed Tabu / local search over vehicle relocations (heterogeneous fleet)."""
    B, M, ldc = _table(C, M)
    dev = C.device
    f, keep = _fleet(K_r, K_f, heliport, rotary_only, dev, B, M)
    K = int(K_r) + int(K_f)
    p = Params(int(tenure), int(iterations), int(range_m), int(mode), int(seed) % 2**64)
    best = torch.empty(K, dtype=torch.int32, device=dev)
    brot = torch.empty(K, dtype=torch.int32, device=dev)
    assign = torch.empty(M, dtype=torch.int32, device=dev) if want_assign else None
    n = max(int(iterations), 0)
    trace = torch.empty(max(n, 1) * TRACE_DTYPE.itemsize, dtype=torch.uint8, device=dev) \
        if want_trace else None
    init = irot = None
    if init_open is not None:
        init = torch.as_tensor(init_open).to(device=dev, dtype=torch.int32).contiguous()
        if init_rotary is not None:
            irot = torch.as_tensor(init_rotary).to(device=dev, dtype=torch.int32).contiguous()
    sc = Score()
    _check(lib().fs_fleet_solve(_table_ptr(C), ldc, B, M, ctypes.byref(f), ctypes.byref(p),
                                _ptr(init), _ptr(irot), _ptr(best), _ptr(brot),
                                ctypes.byref(sc), _ptr(assign),
                                _ptr(trace) if n > 0 else None, _stream(stream)))
    tr = None
    if want_trace:
        tr = trace[: n * TRACE_DTYPE.itemsize].cpu().numpy().view(TRACE_DTYPE)
    return FleetResult(best, int(sc.coverage), int(sc.distance), int(sc.best_iter), assign, tr,
                       brot)


def timing_enable(on: bool = True, every: int = 1) -> None:
    """Time every `every`-th sweep / refresh launch with dispatch-stamped HIP
    events (off with on=False)."""
    _check(lib().fs_timing_enable(int(every) if on else 0))


def timing_read(group: str):
    """(total device ms, launches) recorded for a kernel group since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().fs_timing_read(group.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


@dataclass
class ServeResult:
    best_open: np.ndarray     # host int32 K, ascending
    coverage: int
    distance: int
    best_iter: int
    latency_s: float


class Server:
    """Repositioning server (continuous batching over resident cost tables).
    Coordinates and mission redraws are host arrays (copied by the server)."""

    def __init__(self, hbm_budget_bytes: int = 200 << 30, max_slots: int = 64, device: int = 0,
                 earth_radius_m: float = 0.0, legs: int = 3):
        cfg = ServeConfig(int(hbm_budget_bytes), int(max_slots), int(device),
                          float(earth_radius_m), int(legs), 0)
        h = ctypes.c_void_p()
        _check(lib().fs_serve_open(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._K = {}

    def register(self, bases, missions, K: int, range_m: int) -> int:
        b = np.ascontiguousarray(bases, dtype=np.float64)
        m = np.ascontiguousarray(missions, dtype=np.float64)
        iid = ctypes.c_int64()
        _check(lib().fs_serve_register(self._h, b.ctypes.data, b.shape[0], m.ctypes.data,
                                       m.shape[0], int(K), int(range_m), ctypes.byref(iid)))
        self._K[iid.value] = int(K)
        return int(iid.value)

    def submit(self, instance_id: int, mission_ids, new_pd, tenure: int, iterations: int,
               mode: int = 0, seed: int = 0) -> int:
        ids = np.ascontiguousarray(mission_ids, dtype=np.int32)
        pd = np.ascontiguousarray(new_pd, dtype=np.float64).reshape(-1, 4)
        p = Params(int(tenure), int(iterations), 0, int(mode), int(seed) % 2**64)
        t = ctypes.c_uint64()
        _check(lib().fs_serve_submit(self._h, int(instance_id), ids.ctypes.data if ids.size else None,
                                     pd.ctypes.data if ids.size else None, int(ids.size),
                                     ctypes.byref(p), ctypes.byref(t)))
        return int(t.value), int(instance_id)

    def poll(self, ticket):
        """ServeResult when done, None while pending (ticket is (id, instance))."""
        tk, iid = ticket
        out = np.zeros(self._K[iid], dtype=np.int32)
        sc = Score()
        lat = ctypes.c_double()
        st = lib().fs_serve_poll(self._h, tk, out.ctypes.data, ctypes.byref(sc), ctypes.byref(lat))
        if st == FS_PENDING:
            return None
        _check(st)
        return ServeResult(out, int(sc.coverage), int(sc.distance), int(sc.best_iter),
                           float(lat.value))

    def wait(self, ticket, timeout: float = 120.0, interval: float = 2e-4):
        import time
        t_end = time.monotonic() + timeout
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() > t_end:
                raise TimeoutError(f"request {ticket} not done after {timeout} s")
            time.sleep(interval)

    def stats(self) -> dict:
        st = ServeStats()
        _check(lib().fs_serve_stats_get(self._h, ctypes.byref(st)))
        return {f: int(getattr(st, f)) for f, _ in ServeStats._fields_}

    def close(self):
        if self._h:
            _check(lib().fs_serve_close(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
