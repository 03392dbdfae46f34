"""plbm_reduce_static, the reduction for callers that cannot allocate: its
tile records live in the library's static per-GPU device array instead of the
lattice's buffer.  Its output must equal plbm_reduce's on a twin lattice
(same kernels, same fixed order: bitwise), on consecutive calls with a
smaller lattice second (the array keeps the previous call's records), and a
lattice with more tiles than the array holds is refused with a clear error.
"""
import numpy as np
import pytest

from gpu_cases import fmt, lib_params, random_state, require_gpu

pytestmark = pytest.mark.gpu

FIELDS = ("mass", "mass_comp_err", "max_u", "max_du_per_step", "time", "flags")


def _same(a, b):
    for f in FIELDS:
        assert getattr(a, f) == getattr(b, f), (f, getattr(a, f), getattr(b, f))
    assert list(a.momentum) == list(b.momentum)


def _twins(lattice, dims, storage, collision, pattern, seed):
    from paper_2504_15018_amd.lattice import Lattice
    f0 = random_state(lattice, dims, seed, rel_amp=0.05)
    out = []
    for _ in range(2):
        lat = Lattice(lattice, dims, lib_params(Fg=(1e-5, 0.0, 0.0)), collision=collision, storage=storage,
                      pattern=pattern)
        lat.write_populations(f0)
        out.append(lat)
    return out


def test_static_workspace_reduce_equals_plbm_reduce():
    require_gpu()
    from paper_2504_15018_amd import native as N
    # the larger lattice first, then a smaller one: the second call finds the first one's records in the array
    cases = [("D3Q19", (150, 40, 37), "f32", "mrt", "ab"), ("D2Q9", (70, 33), "f64", "bgk", "aa"),
             ("D3Q19", (20, 9, 5), "f16r", "mrt", "aa")]
    for case in cases:
        fmt("no_alloc_reduce", case=case)
        a, b = _twins(*case, seed=17)
        for k in range(3):
            da = N.plbm_reduce(a.h)
            db = N.plbm_reduce_static(b.h)
            _same(da, db)
            if k:
                assert db.max_du_per_step > 0.0
            a.step(3)
            b.step(3)
        assert np.array_equal(a.populations(), b.populations())
        a.close()
        b.close()


def test_static_workspace_refuses_more_tiles_than_it_holds():
    require_gpu()
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    fmt("no_alloc_limit")
    # one z plane of 256 x 129 tiles of 64 x 8 nodes: 33 024 tiles, one more than 32 767
    lat = Lattice("D3Q19", (16384, 1032, 1), lib_params(), collision="bgk", storage="f32")
    lat.init_shape(N.PLBM_SHAPE_DROPLET, 7.0, 0.25, W=5.0, R=100.0)
    with pytest.raises(N.PlbmError) as e:
        N.plbm_reduce_static(lat.h)
    assert e.value.code == N.PLBM_E_NOMEM and "32767" in str(e.value)
    d = lat.reduce()  # the workspace-in-buffer reduction has no such limit
    assert d.flags == 0 and d.mass > 0
    lat.close()
