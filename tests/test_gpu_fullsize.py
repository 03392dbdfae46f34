"""Parity at the full workload sizes, in the launch configuration the benchmark
times (the lattice's own stream, multi-step calls replayed from a HIP graph).

A time-stepping stencil cannot be sampled one output at a time, but it has a
light cone: one update reads populations one node away and the force at that
node reads psi one node further, so after K steps a node depends only on the
initial state within 2K nodes.  The oracle therefore runs on periodic boxes of
the sampled window plus a 2K margin, cut out of the same host-generated
initial state, and its interior must match the full-size GPU run.  Laterally
uniform problems (the planar slab, the layered channel) are one-dimensional:
every GPU column must equal a single-column oracle run.

Tolerances as in the small-size parity tests: float64 1e-12 relative (f, rho)
and 1e-12 absolute (u); float32 1.5e-6 sqrt(steps) relative and 2e-7
sqrt(steps) absolute (gpu_cases.tols).
"""
import numpy as np
import pytest

import plbm_synth as syn
from oracle import step as S

from gpu_cases import abs_max, fmt, lib_params, oracle_params, rel_max, require_gpu, tols

pytestmark = pytest.mark.gpu


def _tol(storage, steps):
    return tols(storage, steps)


def _window_parity(lat, op, rho_fn, u0, dims, storage, steps, windows, out_size):
    """Compare GPU populations after `steps` with oracle runs on margin-padded windows."""
    f_gpu = lat.populations()
    d = len(dims)
    m = 2 * steps
    tf, tu = _tol(storage, steps)
    for lo in windows:
        box_lo = [l - m for l in lo]
        size = [out_size + 2 * m] * d
        co = syn.window(dims, box_lo, size)
        rho0 = rho_fn(co)
        u = np.zeros((d,) + rho0.shape)
        for a in range(d):
            u[a] = u0[a]
        f0 = S.init_equilibrium(op.lat, rho0, u)
        if storage == "f32":
            f0 = f0.astype(np.float32).astype(np.float64)
        # the box is periodic on the oracle's side only: the density jumps at its
        # seams can overflow the EOS there, outside the light cone of the interior
        with np.errstate(over="ignore", invalid="ignore"):
            ref = S.run(op, f0, steps)
        inner = tuple(slice(m, m + out_size) for _ in range(d))
        ref_in = ref[(slice(None),) + inner]
        # the same nodes of the GPU lattice (arrays are indexed (.., z, y, x))
        idx = tuple(np.ix_(*[(np.arange(out_size) + lo[a]) % dims[a] for a in reversed(range(d))]))
        got = f_gpu[(slice(None),) + idx]
        err = rel_max(got, ref_in)
        fmt("window", lo=lo, rel_f=f"{err:.3e}")
        assert err <= tf, (lo, err)
        with np.errstate(over="ignore", invalid="ignore"):  # the seams again
            rho_r, u_r = S.moments(op, ref)
        rho_g = got.sum(axis=0)
        assert rel_max(rho_g, rho_r[inner]) <= tf
    return f_gpu


@pytest.mark.parametrize("variant", ["static", "galilean", "static-inplace", "static-f64", "galilean-inplace-f64"])
def test_c3_droplet_256cubed_mrt_windows(variant):
    """D3Q19 256^3, float32 MRT + Guo, PR T/Tc = 0.8, droplet R = 48 (W = 5); Galilean variant u0 = 0.05 x;
    the in-place pattern over an odd step count (ends in the odd-time layout); the same in float64 storage
    (`bench.py --storage f64`), at the float64 bar."""
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    fmt("c3_fullsize", variant=variant)
    dims = (256, 256, 256)
    op = oracle_params("D3Q19", collision="mrt")
    rv, rl = op.rho_v, op.rho_l
    u0 = (0.05, 0.0, 0.0) if variant.startswith("galilean") else (0.0, 0.0, 0.0)

    def rho_fn(co):
        return syn.droplet(co, dims, rv, rl, R=48.0, W=5.0)

    co = syn.grid(dims)
    rho_full = rho_fn(co)
    del co
    u_full = np.zeros((3,) + rho_full.shape)
    u_full[0] = u0[0]
    inplace = "inplace" in variant
    storage = "f64" if variant.endswith("f64") else "f32"
    lat = Lattice("D3Q19", dims, lib_params(), collision="mrt", storage=storage, pattern="aa" if inplace else "ab")
    lat.init_fields(rho_full, u_full)
    del u_full
    steps = 13 if inplace else 12
    lat.step(steps)
    windows = [(172, 124, 124), (124, 124, 124), (252, 250, 251), (100, 170, 30)]
    _window_parity(lat, op, rho_fn, u0, dims, storage, steps, windows, 8)
    lat.close()


@pytest.mark.parametrize("tr", [0.7, 0.8, 0.9])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_c2_droplet_512sq_mrt_windows(storage, tr):
    """D2Q9 512^2, MRT, PR at T/Tc in {0.7, 0.8, 0.9}, droplet R = 64 (W = 5), float64 and float32."""
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    fmt("c2_fullsize", storage=storage, tr=tr)
    dims = (512, 512)
    op = oracle_params("D2Q9", tr=tr, collision="mrt")
    rv, rl = op.rho_v, op.rho_l

    def rho_fn(co):
        return syn.droplet(co, dims, rv, rl, R=64.0, W=5.0)

    lat = Lattice("D2Q9", dims, lib_params(tr=tr), collision="mrt", storage=storage)
    lat.init_fields(rho_fn(syn.grid(dims)))
    steps = 40
    lat.step(steps)
    windows = [(312, 248), (248, 248), (500, 505), (290, 290), (40, 400)]
    _window_parity(lat, op, rho_fn, (0.0, 0.0), dims, storage, steps, windows, 16)
    lat.close()


def test_c4_channel_384x384x128_f64_columns_equal_oracle():
    """D3Q19 384x384x128 between half-way bounce-back plates, F_g = 1e-6 x, layered liquid/vapour, BGK
    tau = 1, float64: every column bitwise equal, and equal to the 1x1x128 oracle column."""
    require_gpu()
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    fmt("c4_fullsize_f64")
    dims = (384, 384, 128)
    Fg = (1e-6, 0.0, 0.0)
    op = oracle_params("D3Q19", walls=True, Fg=Fg)
    lat = Lattice("D3Q19", dims, lib_params(Fg=Fg), storage="f64", walls=True)
    lat.init_shape(N.PLBM_SHAPE_LAYERS, op.rho_l, op.rho_v, W=5.0, level=64.0, axis=2)
    steps = 300
    lat.step(steps)
    f = lat.populations()
    assert np.array_equal(f, np.broadcast_to(f[:, :, :1, :1], f.shape))
    col = f[:, :, :1, :1]
    del f
    co1 = syn.grid((1, 1, 128))
    rho0 = syn.layers(co1, (1, 1, 128), op.rho_v, op.rho_l, W=5.0)
    ref = S.run(op, S.init_equilibrium(op.lat, rho0), steps)
    assert rel_max(col, ref) <= 1e-12
    rho, u = lat.moments()
    rho_r, u_r = S.moments(op, ref)
    assert rel_max(rho[:, :1, :1], rho_r) <= 1e-12
    assert abs_max(u[:, :, :1, :1], u_r) <= 1e-12
    lat.close()
