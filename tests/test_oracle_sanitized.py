"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

`tests/oracle_driver.c` calls every exported oracle function on small seeded
instances (padded row pitch, K = 1 and K = B, R = 0, T = 0, N = 0, one mission,
both leg counts, all search modes, the typed fleet, the exhaustive optima) and
prints a digest of each call's outputs.  It is built twice with gcc: plainly,
and with ASan + UBSan (any report aborts the run).  Every run must exit with
status 0 and print the same digests, whatever the OpenMP thread count and
whatever value fills the table's row padding (which no function may read).

A control program with one out-of-bounds read shows that the sanitizer build
does catch such a read on this machine.

ThreadSanitizer: the same driver built by LLVM's clang against LLVM's OpenMP
runtime, with the Archer tool supplying OpenMP's synchronisation to the race
detector (without it every fork and join of a parallel region reads as a
race), at 2, 4 and 8 threads; a control program that increments one variable
from every thread of a parallel region shows that a race is reported.
"""

from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SRCS = [os.path.join(ROOT, "oracle", n)
               for n in ("fleetstage_oracle.c", "fleet_oracle.c", "perm_oracle.c")]
DRIVER = os.path.join(ROOT, "tests", "oracle_driver.c")
COMMON = ["-std=c11", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra"]
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=all"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")


def _gcc(out, srcs, flags):
    cmd = ["gcc", *COMMON, *flags, "-o", str(out), *srcs, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([str(exe), *map(str, args)], capture_output=True, text=True,
                          timeout=300, env=env)


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("sanitized_oracle")
    plain, san = d / "plain", d / "sanitized"
    _gcc(plain, [DRIVER, *ORACLE_SRCS], ["-O2"])
    _gcc(san, [DRIVER, *ORACLE_SRCS], SANITIZE)
    return d, plain, san


def test_sanitizer_catches_an_out_of_bounds_read(builds):
    d, _, _ = builds
    src = d / "control.c"
    src.write_text("#include <stdlib.h>\n"
                   "int main(int argc, char **argv) {\n"
                   "    (void)argv;\n"
                   "    int *a = malloc(4 * sizeof(int));\n"
                   "    for (int i = 0; i < 4; ++i) a[i] = i;\n"
                   "    int v = a[3 + argc];   /* one past the end */\n"
                   "    free(a);\n"
                   "    return v == 12345;\n"
                   "}\n")
    exe = d / "control"
    _gcc(exe, [str(src)], SANITIZE)
    r = _run(exe)
    assert r.returncode != 0
    # UBSan's object-size check or ASan's shadow check, whichever sees it first
    assert "heap-buffer-overflow" in r.stderr or "insufficient space" in r.stderr, r.stderr


def test_oracle_clean_under_sanitizers(builds):
    _, plain, san = builds
    ref = _run(plain, 2, -7)
    assert ref.returncode == 0, ref.stderr
    lines = ref.stdout.splitlines()
    assert len(lines) > 60
    # every function and search mode appears
    for name in ("scalars", "cost_table(3 legs)", "cost_table(2 legs)", "row_sums",
                 "rank_bases", "value+assign", "move_scores", "tabu", "local_search",
                 "perm_local", "perm_tabu", "fleet rank+scores", "fleet_tabu",
                 "fleet_local_search", "brute_optimum", "fleet_brute_optimum"):
        assert any(l.startswith(name + " ") for l in lines), name
    for exe, threads, pad in ((san, 2, -7), (san, 4, 2**31 - 1), (plain, 1, 0),
                              (plain, 8, -(2**31))):
        r = _run(exe, threads, pad)
        assert r.returncode == 0, (exe.name, threads, pad, r.stderr[-4000:])
        assert "runtime error" not in r.stderr, r.stderr[-4000:]
        assert "Sanitizer" not in r.stderr, r.stderr[-4000:]
        assert r.stdout == ref.stdout, (exe.name, threads, pad)


LLVM_BIN = "/opt/rocm/llvm/bin/clang"
LLVM_LIB = "/opt/rocm/llvm/lib"
ARCHER = os.path.join(LLVM_LIB, "libarcher.so")
needs_archer = pytest.mark.skipif(
    not (os.path.exists(LLVM_BIN) and os.path.exists(ARCHER)),
    reason="LLVM clang with the Archer OpenMP tool not found")
TSAN = ["-O1", "-g", "-fsanitize=thread", "-fopenmp", "-Wl,-rpath," + LLVM_LIB]


def _clang(out, srcs):
    cmd = [LLVM_BIN, "-std=c11", "-fno-fast-math", "-ffp-contract=off", *TSAN, "-o", str(out),
           *srcs, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr


def _run_tsan(exe, *args):
    env = dict(os.environ, OMP_TOOL_LIBRARIES=ARCHER,
               TSAN_OPTIONS="ignore_noninstrumented_modules=1")
    env.pop("ARCHER_OPTIONS", None)
    return subprocess.run([str(exe), *map(str, args)], capture_output=True, text=True,
                          timeout=300, env=env)


@needs_archer
def test_thread_sanitizer_catches_a_race(tmp_path):
    src = tmp_path / "race.c"
    src.write_text("#include <stdio.h>\n"
                   "int main(void) {\n"
                   "    int x = 0;\n"
                   "#pragma omp parallel num_threads(4)\n"
                   "    x += 1;   /* every thread, unsynchronised */\n"
                   "    printf(\"%d\\n\", x > 0);\n"
                   "    return 0;\n"
                   "}\n")
    exe = tmp_path / "race"
    _clang(exe, [str(src)])
    r = _run_tsan(exe)
    assert r.returncode != 0
    assert "ThreadSanitizer: data race" in r.stderr, r.stderr


@needs_archer
def test_oracle_clean_under_thread_sanitizer(builds, tmp_path):
    _, plain, _ = builds
    ref = _run(plain, 2, -7)
    assert ref.returncode == 0, ref.stderr
    exe = tmp_path / "tsan"
    _clang(exe, [DRIVER, *ORACLE_SRCS])
    for threads in (2, 4, 8):
        r = _run_tsan(exe, threads, -7)
        assert r.returncode == 0, (threads, r.stderr[-4000:])
        assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
        assert r.stdout == ref.stdout, threads
