"""Helpers shared by the GPU parity tests (no method arithmetic here)."""

import numpy as np
import torch

import oracle
from paper_2001_05291_amd import synth

DEV = "cuda:0"


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def padded_table(C, ldc):
    """Copy of an oracle table into a device tensor of row pitch ldc (the
    padding holds a large poison value the kernels must never read as a cost)."""
    B, M = C.shape
    host = np.full((B, ldc), 2_000_000_000, dtype=np.int32)
    host[:, :M] = C
    return to_dev(host)


def oracle_table(inst):
    C, _ = oracle.cost_table(inst.bases, inst.missions, want_cf=False)
    return C


def assert_trace_equal(gpu_trace, ref, n=None):
    n = len(ref.moved) if n is None else n
    tr = gpu_trace[:n]
    assert np.array_equal(tr["iter"], np.arange(1, n + 1))
    for gname, rname in (("out_base", "out_base"), ("in_base", "in_base"), ("moved", "moved"),
                         ("cur_cov", "cur_cov"), ("cur_dist", "cur_dist"),
                         ("best_cov", "best_cov"), ("best_dist", "best_dist")):
        g = tr[gname]
        r = getattr(ref, rname)[:n]
        if not np.array_equal(g, r):
            bad = int(np.nonzero(g != r)[0][0])
            raise AssertionError(f"trace field {gname} differs first at iteration {bad + 1}: "
                                 f"gpu {g[bad]} oracle {r[bad]}")


def instance_and_table(cfg):
    inst = synth.workload_instance(cfg)
    return inst, oracle_table(inst)
