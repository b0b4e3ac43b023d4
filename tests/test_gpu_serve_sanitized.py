"""The repositioning server's host runtime under AddressSanitizer and
UndefinedBehaviorSanitizer (device code unchanged).

`tests/bin/serve_asan` (built by `tests/sanitized_build.py`, which
`__graft_entry__.build()` runs) drives the server from four client threads and
a counter reader against a budget that forces evictions, compares every result
with a one-slot server, and closes a server with requests in flight
(`tests/serve_driver.cpp`).  The run passes when it exits 0 with no sanitizer
report.  Leaks are checked with the HIP and HSA runtimes' own allocations
suppressed.
"""

from __future__ import annotations

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
BIN = os.path.join(HERE, "bin")

pytestmark = pytest.mark.gpu


def _exe(kind):
    exe = os.path.join(BIN, f"serve_{kind}")
    if not os.path.exists(exe):
        raise FileNotFoundError(f"{exe} is missing: run tests/sanitized_build.py (or "
                                "__graft_entry__.build()) first")
    return exe


def _check(r):
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stderr[-6000:]
    for mark in ("ERROR: AddressSanitizer", "runtime error:",
                 "ERROR: LeakSanitizer"):
        assert mark not in r.stderr, r.stderr[-6000:]
    assert "0 mismatches" in r.stdout


def test_serve_under_address_sanitizer(tmp_path):
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64.so\nleak:libhsa-runtime64.so\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:exitcode=66",
               LSAN_OPTIONS=f"suppressions={supp}",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([_exe("asan")], capture_output=True, text=True, timeout=300, env=env)
    _check(r)
