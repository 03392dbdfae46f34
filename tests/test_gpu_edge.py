"""Edge cases of the HIP path (through the C ABI).

* Degenerate shapes against the FP64 oracle: extents of 1 and 2 (a node is its
  own periodic neighbour), a single plane between two walls, lattices smaller
  than one tile, in both storage patterns; float64 bar 1e-12, float32 gpu_cases.tols per
  step (as the other parity tests).
* Zero steps change nothing.

The largest accepted lattice is exercised in test_gpu_zz_largest.py (it runs
last: it needs about 190 GB of HBM).
"""
import numpy as np
import pytest

from oracle import step as S

from gpu_cases import abs_max, fmt, lib_params, oracle_params, rel_max, random_state, require_gpu, tols

pytestmark = pytest.mark.gpu

SHAPES = [
    # lattice, dims, collision, storage, walls, pattern, steps
    ("D3Q19", (1, 1, 1), "bgk", "f64", False, "ab", 3),
    ("D3Q19", (1, 1, 5), "mrt", "f64", True, "aa", 4),
    ("D3Q19", (2, 3, 1), "mrt", "f64", False, "ab", 3),
    ("D3Q19", (3, 1, 4), "mrt", "f64", True, "ab", 5),
    ("D3Q19", (5, 4, 1), "bgk", "f64", True, "aa", 3),  # one plane between two walls
    ("D3Q19", (65, 9, 2), "mrt", "f32", True, "aa", 3),
    ("D3Q19", (7, 2, 2), "bgk", "f32", False, "ab", 4),
    ("D2Q9", (1, 9), "mrt", "f64", False, "ab", 4),
    ("D2Q9", (7, 1), "bgk", "f64", True, "aa", 3),  # one row between two walls
    ("D2Q9", (1, 1), "bgk", "f64", False, "aa", 2),
    ("D2Q9", (129, 2), "mrt", "f64", True, "ab", 5),
]


@pytest.mark.parametrize("case", SHAPES, ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[1]))}-{c[2]}-{c[3]}-"
                                                         f"{'bb' if c[4] else 'per'}-{c[5]}")
def test_degenerate_shapes_match_the_oracle(case):
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    lattice, dims, collision, storage, walls, pattern, steps = case
    fmt("edge_shape", case=case)
    f0 = random_state(lattice, dims, 23)
    op = oracle_params(lattice, collision=collision, walls=walls)
    lat = Lattice(lattice, dims, lib_params(), collision=collision, storage=storage, walls=walls, pattern=pattern)
    lat.write_populations(f0)
    if storage == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    assert np.array_equal(lat.populations(), f0)
    lat.step(steps)
    f_ref = S.run(op, f0, steps)
    tf, tu = tols(storage, steps)
    assert rel_max(lat.populations(), f_ref) <= tf
    rho, u = lat.moments()
    rho_ref, u_ref = S.moments(op, f_ref)
    assert rel_max(rho, rho_ref) <= tf
    assert abs_max(u, u_ref) <= tu
    d = lat.reduce()
    # the +-30 % random states reach 1.3 rho_l, where the psi radicand can turn negative (clamped on both sides,
    # PSI_NEG raised): only NaN and rho <= 0 are failures here
    assert not (d.flags & 3) and d.time == steps
    lat.close()


@pytest.mark.parametrize("pattern", ["ab", "aa"])
def test_zero_steps_change_nothing(pattern):
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    fmt("edge_zero_steps", pattern=pattern)
    dims = (33, 17, 9)
    f0 = random_state("D3Q19", dims, 2)
    lat = Lattice("D3Q19", dims, lib_params(), collision="mrt", storage="f64", pattern=pattern)
    lat.write_populations(f0)
    lat.step(0)
    assert lat.time == 0 and np.array_equal(lat.populations(), f0)
    lat.step(3)
    f3 = lat.populations()
    lat.step(0)
    assert lat.time == 3 and np.array_equal(lat.populations(), f3)
    lat.close()


SHORT_AXES = [
    # lattice, dims (the last axis is the kernel's marching axis), steps
    ("D3Q19", (5, 3, 1), 3),
    ("D3Q19", (5, 3, 2), 3),
    ("D3Q19", (4, 3, 3), 4),
    ("D2Q9", (7, 1), 3),
    ("D2Q9", (7, 2), 4),
]


@pytest.mark.parametrize("pattern", ["ab", "aa"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s", "f16r", "bf16r"])
@pytest.mark.parametrize("case", SHORT_AXES, ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[1]))}")
def test_short_periodic_marching_axis_reads_stay_inside_the_lattice(case, storage, pattern):
    """A periodic marching axis shorter than the march's load window (one to
    three planes) must wrap inside the population arrays (both patterns: the
    in-place update loads the psi ring a plane ahead).  The lattice sits at
    the start of a buffer whose remaining megabyte holds all-ones bytes (NaN
    in every storage format): a load past the lattice's own bytes would sum a
    NaN density, whose psi radicand raises the PSI_NEG flag of the reduction
    (and NaN populations would break parity).  The state is a smooth +-5 %
    perturbation, far from the densities where the radicand turns negative,
    so any flag is a read outside the lattice."""
    require_gpu()
    import torch

    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import make_desc
    from oracle.lattice import LATTICES
    from gpu_cases import ULP, storage_round

    lattice, dims, steps = case
    fmt("edge_short_axis", case=case, storage=storage, pattern=pattern)
    op = oracle_params(lattice, collision="mrt")
    rl = op.rho_l
    shifted = storage in ("f16s", "bf16s")
    desc = make_desc(lattice, dims, "mrt", storage, rho0_shift=rl if shifted else 0.0, pattern=pattern)
    nb = N.plbm_lattice_bytes(desc)
    pad = 1 << 20
    mem = torch.full((nb + 256 + pad,), 0xFF, dtype=torch.uint8, device="cuda")
    ptr = (mem.data_ptr() + 255) // 256 * 256
    stream = torch.cuda.Stream()
    h = N.plbm_create(desc, lib_params(), ptr, nb, stream.cuda_stream)
    Q = LATTICES[lattice].Q
    n = int(np.prod(dims))
    try:
        f_in = random_state(lattice, dims, 31, rel_amp=0.05)
        N.plbm_write_populations(h, f_in.reshape(-1))
        f0 = f_in if storage == "f64" else (f_in.astype(np.float32).astype(np.float64) if storage == "f32"
                                            else storage_round(lattice, f_in, storage, rl))
        ref = f0
        for k in range(steps):
            d = N.plbm_reduce(h, True)  # both time parities
            assert d.flags == 0, (k, d.flags)
            N.plbm_step(h, 1)
            ref = S.step(op, ref)
        d = N.plbm_reduce(h, True)
        assert d.flags == 0, d.flags
        f = N.plbm_read_populations(h, Q, n).reshape(ref.shape)
        if storage == "f64":
            tol = 1e-12
        elif storage == "f32":
            tol = tols(storage, steps)[0]
        else:
            w = LATTICES[lattice].w.reshape((-1,) + (1,) * len(dims))
            dev = np.max(np.abs(ref - w * (rl if shifted else ref.sum(axis=0)[None])))
            tol = steps * (ULP[storage] * dev / np.max(np.abs(ref)) + 2e-6)
        err = rel_max(f, ref)
        fmt("edge_short_axis_err", err=f"{err:.3e}", tol=f"{tol:.3e}")
        assert err <= tol
        # the bytes after the lattice are untouched
        stream.synchronize()
        tail = mem[ptr - mem.data_ptr() + nb:]
        assert bool((tail == 0xFF).all())
    finally:
        stream.synchronize()
        N.plbm_destroy(h)
