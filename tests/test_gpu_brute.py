"""GPU parity of the exact optimum by enumeration (the stand-in for the
paper's exact-solver column, Section 5): the HIP path through the C ABI
against the CPU oracle's enumeration, bit for bit (placement, value, count)."""

import numpy as np
import pytest
import torch

import oracle
from paper_2001_05291_amd import synth

pytestmark = pytest.mark.gpu

from gpu_util import instance_and_table, padded_table  # noqa: E402

fs = None


@pytest.fixture(scope="module", autouse=True)
def _lib():
    global fs
    from paper_2001_05291_amd import fleetstage
    fs = fleetstage
    fs.lib()
    torch.cuda.init()
    yield


def check(C, K, R, ldc=None):
    B, M = C.shape
    best, cov, dist, n = fs.brute_optimum(padded_table(C, ldc or M), K, R, M=M)
    o_best, o_cov, o_dist, o_n = oracle.brute_optimum(C, K, R)
    assert np.array_equal(best.cpu().numpy(), o_best)
    assert (cov, dist, n) == (o_cov, o_dist, o_n)
    return cov, dist


def test_small_workload():
    c = synth.WORKLOADS["small"]
    _, C = instance_and_table("small")
    cov, dist = check(C, c["K"], c["R"])
    t = fs.tabu_solve(padded_table(C, C.shape[1]), c["K"], c["R"], c["T"], c["N"])
    assert (t.coverage, -t.distance) <= (cov, -dist)


def test_random_tables_with_ties_and_edges():
    rng = np.random.default_rng(17)
    for trial in range(40):
        B = int(rng.integers(1, 26))
        M = int(rng.integers(1, 120))
        K = int(rng.integers(1, min(B, 6) + 1))
        hi = 4 if trial % 3 == 0 else 3000       # many equal values
        C = rng.integers(1, hi, size=(B, M)).astype(np.int32)
        R = int(rng.integers(0, hi + 100))
        check(C, K, R, ldc=M + int(rng.integers(0, 5)))


def test_all_bases_and_single_vehicle():
    rng = np.random.default_rng(5)
    C = rng.integers(1, 1000, size=(9, 50)).astype(np.int32)
    check(C, 9, 700)
    check(C, 1, 700)
    check(C, 5, 0)


def test_enumeration_limits_are_errors():
    C = padded_table(np.ones((100, 200), dtype=np.int32), 200)
    with pytest.raises(fs.FleetstageError) as e:       # table too large to stage
        fs.brute_optimum(C, 3, 10)
    assert e.value.status == fs.FS_E_INVALID
    C = padded_table(np.ones((60, 10), dtype=np.int32), 10)
    with pytest.raises(fs.FleetstageError) as e:       # C(60, 17): K too large
        fs.brute_optimum(C, 17, 10)
    assert e.value.status == fs.FS_E_INVALID
