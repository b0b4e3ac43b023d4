"""The indexed cost-table builder (missions as hospital-id pairs): bitwise the
direct builder's table and FP64 sums, and within the oracle's tolerance
(Eq. 1; Section 3 mission legs)."""

import numpy as np
import pytest
import torch

import oracle
from paper_2001_05291_amd import synth

pytestmark = pytest.mark.gpu

from gpu_util import to_dev  # noqa: E402

fs = None


@pytest.fixture(scope="module", autouse=True)
def _lib():
    global fs
    from paper_2001_05291_amd import fleetstage
    fs = fleetstage
    fs.lib()
    torch.cuda.init()
    yield


def both(inst, legs=3, ldc=None):
    Cd, Cfd = fs.build_cost_table(to_dev(inst.bases), to_dev(inst.missions), legs=legs, ldc=ldc,
                                  want_cf=True)
    Ci, Cfi = fs.build_cost_table_indexed(to_dev(inst.bases), to_dev(inst.hospitals),
                                          to_dev(inst.mission_ph), legs=legs, ldc=ldc,
                                          want_cf=True)
    return (Cd.cpu().numpy(), Cfd.cpu().numpy()), (Ci.cpu().numpy(), Cfi.cpu().numpy())


@pytest.mark.parametrize("name", ["small", "medium"])
def test_bitwise_equal_to_direct_form_and_oracle(name):
    inst = synth.workload_instance(name)
    (Cd, Cfd), (Ci, Cfi) = both(inst)
    assert np.array_equal(Ci, Cd)
    assert np.array_equal(Cfi.view(np.int64), Cfd.view(np.int64))
    Co, Cfo = oracle.cost_table(inst.bases, inst.missions)
    assert (np.abs(Cfi - Cfo) / np.maximum(Cfo, 1.0)).max() <= 1e-12
    mism = np.nonzero(Ci != Co)
    for b, m in zip(*mism):
        assert abs(int(Ci[b, m]) - int(Co[b, m])) == 1
        frac = Cfo[b, m] - np.floor(Cfo[b, m])
        assert abs(frac - 0.5) <= 1e-12 * Cfo[b, m] + 1e-9


def test_two_legs_pitch_and_many_hospitals():
    inst = synth.make_instance(seed=61, B=37, H=16_384, M=2003)
    for legs, ldc in ((3, 2008), (2, 2003)):
        (Cd, Cfd), (Ci, Cfi) = both(inst, legs=legs, ldc=ldc)
        assert np.array_equal(Ci, Cd)
        assert np.array_equal(Cfi.view(np.int64), Cfd.view(np.int64))


@pytest.mark.parametrize("H", [10_240, 10_241])
def test_workgroup_size_boundary(H):
    # the largest hospital count whose legs fit two workgroups in a CU's LDS
    # (768-thread workgroups) and the smallest that does not (1,024 threads)
    inst = synth.make_instance(seed=63, B=23, H=H, M=1501)
    (Cd, Cfd), (Ci, Cfi) = both(inst, ldc=1504)
    assert np.array_equal(Ci, Cd)
    assert np.array_equal(Cfi.view(np.int64), Cfd.view(np.int64))


def test_bad_ids_and_too_many_hospitals_are_errors():
    inst = synth.make_instance(seed=62, B=5, H=30, M=40)
    ph = inst.mission_ph.copy()
    ph[7, 1] = 30                     # outside [0, H)
    with pytest.raises(fs.FleetstageError) as e:
        fs.build_cost_table_indexed(to_dev(inst.bases), to_dev(inst.hospitals), to_dev(ph))
    assert e.value.status == fs.FS_E_INVALID
    big = np.zeros((16_385, 2))
    with pytest.raises(fs.FleetstageError) as e:
        fs.build_cost_table_indexed(to_dev(inst.bases), to_dev(big), to_dev(inst.mission_ph))
    assert e.value.status == fs.FS_E_INVALID
