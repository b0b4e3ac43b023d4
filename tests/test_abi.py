"""The C-ABI library loads and exports every entry point declared in
include/*.h.  No compute call is made (CPU only)."""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2001_05291_amd", "libfleetstage.so")


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(fs_\w+)\s*\(", text, re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("fs_build_cost_table", "fs_rank_bases", "fs_move_scores", "fs_tabu_solve",
                     "fs_tabu_solve_batch", "fs_fleet_move_scores", "fs_fleet_solve",
                     "fs_last_error", "fs_version"):
        assert required in names


@pytest.fixture(scope="module")
def library():
    if not os.path.exists(LIB):
        from paper_2001_05291_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(library):
    missing = [n for n in declared_symbols() if not hasattr(library, n)]
    assert not missing, missing


def test_version_and_validation_without_gpu(library):
    library.fs_version.restype = ctypes.c_char_p
    assert b"gfx950" in library.fs_version()
    # argument validation happens on the host before any device call
    library.fs_rank_bases.restype = ctypes.c_int32
    library.fs_rank_bases.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    rc = library.fs_rank_bases(None, 10, 5, 10, 2, None, None, None, None)
    assert rc == -1
    library.fs_last_error.restype = ctypes.c_char_p
    assert b"NULL" in library.fs_last_error()


def test_server_config_validated_before_device_use(library):
    class Cfg(ctypes.Structure):
        _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                    ("device", ctypes.c_int32), ("earth_radius_m", ctypes.c_double),
                    ("legs", ctypes.c_int32), ("pad", ctypes.c_int32)]
    library.fs_serve_open.restype = ctypes.c_int32
    library.fs_serve_open.argtypes = [ctypes.POINTER(Cfg), ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    for cfg in (Cfg(1 << 30, 0, 0, 0.0, 3, 0), Cfg(0, 4, 0, 0.0, 3, 0),
                Cfg(1 << 30, 4, 0, 0.0, 5, 0), Cfg(1 << 30, 4, -1, 0.0, 3, 0)):
        assert library.fs_serve_open(ctypes.byref(cfg), ctypes.byref(h)) == -1


def test_fleet_calls_validated_before_device_use(library):
    vp = ctypes.c_void_p
    library.fs_fleet_solve.restype = ctypes.c_int32
    library.fs_fleet_solve.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32] + \
        [vp] * 10
    assert library.fs_fleet_solve(None, 10, 5, 10, *([None] * 10)) == -1
    library.fs_last_error.restype = ctypes.c_char_p
    assert b"NULL" in library.fs_last_error()
    library.fs_fleet_move_scores.restype = ctypes.c_int32
    library.fs_fleet_move_scores.argtypes = [vp, ctypes.c_int64, ctypes.c_int32,
                                             ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp,
                                             vp, vp]
    assert library.fs_fleet_move_scores(None, 10, 5, 10, None, None, None, 5, None, None,
                                        None) == -1
    assert b"fleet" in library.fs_last_error()
