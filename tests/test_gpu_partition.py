"""Work partition of the update kernels along the marching axis.

A lattice with more tile columns than the device holds workgroups is split in
two classes of work items: whole columns for the first multiple of the resident
workgroup count, shorter chunks for the rest.  Every node's arithmetic is the
same whatever chunk it falls in (the psi planes a chunk recomputes at its ends
are the same values), so populations and moments equal those of the uniform
partition (PLBM_UNIFORM_CHUNKS=1) bitwise; the compensated mass sum and the
maximum speed are reduced in another grouping and agree to rounding.
Both storage patterns, with and without walls, and a batch launch.
"""
import os

import numpy as np
import pytest

from gpu_cases import fmt, lib_params, random_state, require_gpu

pytestmark = pytest.mark.gpu

CASES = [
    # dims, storage, walls, pattern: 288 (f32, 64 x 8 tiles) or 576 (f64, 64 x 4) tile columns
    ((384, 384, 24), "f32", True, "ab"),
    ((384, 384, 24), "f32", False, "aa"),
    ((384, 384, 13), "f64", True, "ab"),
    ((384, 384, 13), "bf16r", False, "aa"),
]


def _make(dims, storage, walls, pattern, uniform, stream=None):
    from paper_2504_15018_amd.lattice import Lattice
    old = os.environ.get("PLBM_UNIFORM_CHUNKS")
    os.environ["PLBM_UNIFORM_CHUNKS"] = "1" if uniform else "0"
    try:
        return Lattice("D3Q19", dims, lib_params(tau_v=0.9, tau_l=1.1, Fg=(1e-5, 0.0, 0.0)), collision="mrt",
                       storage=storage, walls=walls, pattern=pattern, stream=stream)
    finally:
        if old is None:
            del os.environ["PLBM_UNIFORM_CHUNKS"]
        else:
            os.environ["PLBM_UNIFORM_CHUNKS"] = old


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}-{c[1]}-{'bb' if c[2] else 'per'}-{c[3]}")
def test_two_class_partition_equals_uniform(case):
    require_gpu()
    dims, storage, walls, pattern = case
    fmt("partition", case=case)
    f0 = random_state("D3Q19", dims, 31)
    a = _make(dims, storage, walls, pattern, uniform=False)
    b = _make(dims, storage, walls, pattern, uniform=True)
    for lat in (a, b):
        lat.write_populations(f0)
        lat.step(3)
    assert np.array_equal(a.populations(), b.populations())
    ra, ua = a.moments()
    rb, ub = b.moments()
    assert np.array_equal(ra, rb) and np.array_equal(ua, ub)
    for lat in (a, b):
        lat.step(10)  # the graph path
    assert np.array_equal(a.populations(), b.populations())
    da, db = a.reduce(), b.reduce()
    assert abs(da.mass - db.mass) <= 1e-14 * abs(db.mass)
    assert da.max_u == db.max_u and da.flags == db.flags
    a.close()
    b.close()


def test_two_class_partition_in_a_batch():
    require_gpu()
    import torch
    from test_gpu_batch import Batch
    fmt("partition_batch")
    dims = (384, 384, 16)
    stream = torch.cuda.Stream()
    f0 = random_state("D3Q19", dims, 32)
    solo = _make(dims, "f32", True, "ab", uniform=True)
    mixed = _make(dims, "f32", True, "ab", uniform=False, stream=stream)
    small = _make((40, 24, 18), "f32", False, "aa", uniform=False, stream=stream)
    for lat in (solo, mixed):
        lat.write_populations(f0)
    small.write_populations(random_state("D3Q19", (40, 24, 18), 33))
    bt = Batch(2, 1 << 16, stream)
    bt.attach(mixed)
    bt.attach(small)
    bt.step(5)
    stream.synchronize()
    bt.close()
    solo.step(5)
    assert np.array_equal(mixed.populations(), solo.populations())
    for lat in (solo, mixed, small):
        lat.close()
