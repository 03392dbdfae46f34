"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars (stated per quantity, f = post-streaming populations):
  float64 storage: max|df| / max|f| <= 1e-12, max|drho| / max|rho| <= 1e-12,
                   max|du| <= 1e-12 absolute (lattice units);
  float32 storage: max|df| / max|f| <= 1.5e-6 sqrt(steps) (float32 rounding
                   of ~20-operation chains per step, independent from step to
                   step), max|du| <= 2e-7 sqrt(steps) (gpu_cases.tols).
Sizes span several tiles plus ragged tails in every axis.
"""
import numpy as np
import pytest

import plbm_synth as syn
from oracle import diag as OD
from oracle import step as S
from oracle.lattice import LATTICES

from gpu_cases import abs_max, fmt, lib_params, oracle_params, random_state, rel_max, require_gpu, tols

pytestmark = pytest.mark.gpu

def _tols(storage, steps):
    return tols(storage, steps)


CASES = [
    # lattice, dims, collision, storage, walls, steps, extra
    ("D2Q9", (37, 29), "bgk", "f64", False, 6, {}),
    ("D2Q9", (150, 21), "mrt", "f64", True, 6, {"tau_v": 0.8, "tau_l": 1.3, "Fg": (2e-5, -1e-5)}),
    ("D2Q9", (131, 67), "mrt", "f64", False, 5, {"kappa": 1.6}),
    ("D2Q9", (200, 9), "bgk", "f32", True, 5, {"Fg": (1e-5, 0.0)}),
    ("D3Q19", (37, 21, 13), "bgk", "f64", False, 4, {}),
    ("D3Q19", (40, 18, 11), "mrt", "f64", True, 4, {"tau_v": 0.8, "tau_l": 1.2, "Fg": (1e-5, 2e-6, -3e-6)}),
    ("D3Q19", (33, 35, 9), "mrt", "f64", False, 3, {"kappa": 0.7, "tau_v": 1.1, "tau_l": 0.9}),
    ("D3Q19", (35, 17, 10), "mrt", "f32", False, 3, {}),
    ("D3Q19", (32, 16, 12), "bgk", "f32", True, 3, {"Fg": (1e-5, 0.0, 0.0)}),
    ("D2Q9", (64, 40), "mrt", "f64", False, 5, {"eps": 1.3, "kappa": 1.4}),
    ("D3Q19", (33, 18, 11), "bgk", "f64", True, 4, {"eps": 1.0}),
]


def _ids(c):
    return f"{c[0]}-{'x'.join(map(str, c[1]))}-{c[2]}-{c[3]}-{'bb' if c[4] else 'per'}"


def _run_pair(lattice, dims, collision, storage, walls, steps, extra, seed=3):
    from paper_2504_15018_amd.lattice import Lattice
    f0 = random_state(lattice, dims, seed)
    op = oracle_params(lattice, collision=collision, walls=walls, **extra)
    lp = lib_params(**{k: v for k, v in extra.items()})
    lat = Lattice(lattice, dims, lp, collision=collision, storage=storage, walls=walls)
    lat.write_populations(f0)
    if storage == "f32":
        # the oracle starts from the state as rounded into float32 storage,
        # rounded here on the host (round to nearest even, as the encoder)
        f0 = f0.astype(np.float32).astype(np.float64)
        assert np.array_equal(lat.populations(), f0)
    lat.step(steps)
    f_ref = S.run(op, f0, steps)
    return lat, op, f_ref


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_step_parity(case):
    require_gpu()
    lattice, dims, collision, storage, walls, steps, extra = case
    fmt("step_parity", case=_ids(case))
    lat, op, f_ref = _run_pair(*case)
    tf, tu = _tols(storage, steps)
    f = lat.populations()
    assert f.shape == f_ref.shape
    rho, u = lat.moments()
    rho_ref, u_ref = S.moments(op, f_ref)
    fmt("step_parity_err", rel_f=f"{rel_max(f, f_ref):.2e}", rel_rho=f"{rel_max(rho, rho_ref):.2e}",
        abs_u=f"{abs_max(u, u_ref):.2e}", steps=steps)
    assert rel_max(f, f_ref) <= tf
    assert rel_max(rho, rho_ref) <= tf
    assert abs_max(u, u_ref) <= tu
    lat.close()


@pytest.mark.parametrize("case", [c for c in CASES if c[3] == "f64"], ids=_ids)
def test_reduction_parity(case):
    require_gpu()
    fmt("reduction_parity", case=_ids(case))
    lat, op, f_ref = _run_pair(*case)
    d = lat.reduce()
    ref, _ = OD.reduce(op, f_ref)
    assert d.mass == pytest.approx(ref["mass"], rel=1e-14)
    for a in range(lat.D):
        assert d.momentum[a] == pytest.approx(ref["momentum"][a], rel=1e-11, abs=1e-12)
    assert d.max_u == pytest.approx(ref["max_u"], rel=1e-11, abs=1e-13)
    assert d.flags == ref["flags"] == 0
    assert d.time == case[5]
    lat.close()


@pytest.mark.parametrize("lattice,dims", [("D2Q9", (45, 31)), ("D3Q19", (34, 19, 12))])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_init_fields_is_the_equilibrium(lattice, dims, storage):
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    fmt("init_fields", lattice=lattice, storage=storage)
    lat_o = LATTICES[lattice]
    co = syn.grid(dims)
    rho0 = syn.perturb(syn.droplet(co, dims, 0.25, 7.0, R=8.0), co, dims, 5, 0.05)
    u0 = syn.random_velocity(co, dims, 6, 0.05)
    lat = Lattice(lattice, dims, lib_params(), storage=storage)
    lat.init_fields(rho0, u0)
    f = lat.populations()
    ref = S.init_equilibrium(lat_o, rho0, u0)
    assert rel_max(f, ref) <= (2e-16 * 8 if storage == "f64" else 1e-7)
    lat.close()


@pytest.mark.parametrize("lattice,dims,walls", [("D2Q9", (40, 33), True), ("D3Q19", (30, 20, 14), False)])
def test_init_shape_matches_host_fields(lattice, dims, walls):
    require_gpu()
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    fmt("init_shape", lattice=lattice)
    co = syn.grid(dims)
    R = 7.5
    rho0 = syn.droplet(co, dims, 0.2, 7.1, R=R, W=5.0)
    a = Lattice(lattice, dims, lib_params(), walls=walls)
    b = Lattice(lattice, dims, lib_params(), walls=walls)
    a.init_fields(rho0)
    b.init_shape(N.PLBM_SHAPE_DROPLET, 7.1, 0.2, W=5.0, R=R)
    assert rel_max(b.populations(), a.populations()) <= 1e-14
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
def test_write_read_roundtrip(storage):
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    fmt("roundtrip", storage=storage)
    dims = (23, 17, 9)
    f0 = random_state("D3Q19", dims, 11)
    lat = Lattice("D3Q19", dims, lib_params(), storage=storage, walls=True)
    lat.write_populations(f0)
    f = lat.populations()
    if storage == "f64":
        assert np.array_equal(f, f0)
    else:
        # storage rounding only: float32 2^-24, shifted half 2^-11 and bfloat16 2^-8 of |f - w rho0|
        tol = {"f32": 6e-8, "f16s": 5e-4 * 8, "bf16s": 4e-3 * 8}[storage]
        assert rel_max(f, f0) <= tol
        lat.write_populations(f)
        assert np.array_equal(lat.populations(), f)  # idempotent on representable values
    lat.close()


def test_checkpoint_restart_is_bitwise():
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    fmt("checkpoint")
    dims = (41, 22, 10)
    f0 = random_state("D3Q19", dims, 21)
    a = Lattice("D3Q19", dims, lib_params(tau_v=0.9, tau_l=1.1), collision="mrt")
    a.write_populations(f0)
    a.step(7)
    ck = a.populations()
    a.step(5)
    b = Lattice("D3Q19", dims, lib_params(tau_v=0.9, tau_l=1.1), collision="mrt")
    b.write_populations(ck)
    b.step(5)
    assert np.array_equal(a.populations(), b.populations())
    a.close()
    b.close()


def test_rerun_is_bitwise_deterministic():
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    fmt("determinism")
    dims = (70, 37, 19)
    f0 = random_state("D3Q19", dims, 31)
    outs = []
    for _ in range(2):
        lat = Lattice("D3Q19", dims, lib_params(), collision="mrt", storage="f32")
        lat.write_populations(f0)
        lat.step(20)
        outs.append((lat.populations(), lat.reduce().mass))
        lat.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


def test_planar_c1_lateral_invariance_and_oracle():
    """256 x 4 periodic slab (PR T/Tc = 0.8): every column bitwise equal and equal to the 256 x 1 oracle."""
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    fmt("c1_lateral")
    op = oracle_params("D2Q9")
    rv, rl = op.rho_v, op.rho_l
    dims = (256, 4)
    co = syn.grid(dims)
    rho0 = syn.slab(co, dims, rv, rl, W=5.0, axis=0)
    lat = Lattice("D2Q9", dims, lib_params())
    lat.init_fields(rho0)
    d0 = lat.reduce()
    steps = 5000
    lat.step(steps)
    f = lat.populations()
    for y in range(1, 4):
        assert np.array_equal(f[:, y, :], f[:, 0, :])
    co1 = syn.grid((256, 1))
    ref = S.run(op, S.init_equilibrium(op.lat, syn.slab(co1, (256, 1), rv, rl, W=5.0, axis=0)), steps)
    assert rel_max(f[:, :1, :], ref) <= 1e-12
    rho, u = lat.moments()
    rho_ref, u_ref = S.moments(op, ref)
    assert rel_max(rho[:1], rho_ref) <= 1e-12 and abs_max(u[:, :1], u_ref) <= 1e-12
    # coexistence densities (bulk vapour at x = 0, bulk liquid at x = 128) and mass
    assert abs(rho[0, 0] - rho_ref[0, 0]) <= 1e-12 * rho_ref[0, 0]
    assert abs(rho[0, 128] - rho_ref[0, 128]) <= 1e-12 * rho_ref[0, 128]
    d = lat.reduce()
    # mass is conserved up to float64 rounding of the collision (drift ~3e-13 here)
    assert abs(d.mass - d0.mass) <= 1e-12 * d0.mass
    assert abs(d.mass - 4 * OD.reduce(op, ref)[0]["mass"]) <= 1e-12 * d.mass
    lat.close()


def test_graph_replay_matches_single_launches():
    require_gpu()
    import os
    from paper_2504_15018_amd.lattice import Lattice
    fmt("graph_vs_launch")
    dims = (64, 40, 24)
    f0 = random_state("D3Q19", dims, 41)
    a = Lattice("D3Q19", dims, lib_params(), collision="mrt", storage="f32")
    a.write_populations(f0)
    a.step(3)
    a.step(16)  # graph path (odd start)
    b = Lattice("D3Q19", dims, lib_params(), collision="mrt", storage="f32")
    b.write_populations(f0)
    for _ in range(19):
        b.step(1)  # single launches
    assert a.time == b.time == 19
    assert np.array_equal(a.populations(), b.populations())
    a.close()
    b.close()


def test_c3_64cubed_200_steps_against_the_oracle():
    """The C3 problem at 64^3 (droplet R = 12, W = 5, float32 MRT + Guo, Peng-Robinson T/Tc = 0.8) for 200
    steps against the FP64 oracle, at the float32 bars (1.5e-6 sqrt(200) = 2.1e-5 relative on f and rho, 2.8e-6
    absolute on u)."""
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    fmt("c3_64cubed_200")
    n, steps = 64, 200
    dims = (n, n, n)
    op = oracle_params("D3Q19", collision="mrt")
    co = syn.grid(dims)
    rho0 = syn.droplet(co, dims, op.rho_v, op.rho_l, R=12.0, W=5.0)
    lat = Lattice("D3Q19", dims, lib_params(), collision="mrt", storage="f32")
    lat.init_fields(rho0)
    f0 = lat.populations()  # the float32 equilibrium as stored: the oracle starts from the same values
    lat.step(steps)
    f_ref = S.run(op, f0, steps)
    tf, tu = tols("f32", steps)
    f = lat.populations()
    err = rel_max(f, f_ref)
    rho, u = lat.moments()
    rho_ref, u_ref = S.moments(op, f_ref)
    fmt("c3_64cubed_200_err", rel_f=f"{err:.2e}", rel_rho=f"{rel_max(rho, rho_ref):.2e}",
        abs_u=f"{abs_max(u, u_ref):.2e}")
    assert err <= tf
    assert rel_max(rho, rho_ref) <= tf
    assert abs_max(u, u_ref) <= tu
    lat.close()


@pytest.mark.parametrize("lattice,dims,walls", [("D2Q9", (70, 37), True), ("D3Q19", (37, 21, 13), False)])
def test_custom_mrt_rates_match_the_oracle(lattice, dims, walls):
    """plbm_lattice_desc.mrt_rates = (s_e, s_eps, s_q, s_m), four distinct values, float64 (bar 1e-12): a swapped
    or dropped rate class fails."""
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    fmt("custom_mrt_rates", lattice=lattice)
    rates = (1.3, 0.7, 1.5, 0.9)
    f0 = random_state(lattice, dims, 13)
    op = oracle_params(lattice, collision="mrt", walls=walls, tau_v=0.9, tau_l=1.2,
                       rates={"e": rates[0], "eps": rates[1], "q": rates[2], "m": rates[3], "j": 1.0, "rho": 1.0})
    lat = Lattice(lattice, dims, lib_params(tau_v=0.9, tau_l=1.2), collision="mrt", storage="f64", walls=walls,
                  mrt_rates=rates)
    lat.write_populations(f0)
    lat.step(4)
    f_ref = S.run(op, f0, 4)
    assert rel_max(lat.populations(), f_ref) <= 1e-12
    # and the defaults differ measurably, so the rates are really in effect
    op_default = oracle_params(lattice, collision="mrt", walls=walls, tau_v=0.9, tau_l=1.2)
    assert rel_max(S.run(op_default, f0, 4), f_ref) > 1e-6
    lat.close()


@pytest.mark.parametrize("lattice,dims,collision,storage", [("D2Q9", (70, 37), "bgk", "f64"),
                                                            ("D3Q19", (37, 21, 13), "mrt", "f64"),
                                                            ("D3Q19", (35, 17, 10), "mrt", "f32")])
def test_paper_eos_step_matches_the_oracle(lattice, dims, collision, storage):
    """The paper's own EOS (eq. EOS with K from eq. thickness; R134a-like lattice densities 0.0375 / 1.187,
    interface width xi = 3) stepped against the oracle, on the usual float64 / float32 bars."""
    require_gpu()
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    from oracle import eos as E
    fmt("paper_eos_parity", lattice=lattice, storage=storage)
    rv, rl, xi = 0.0375, 1.187, 3.0
    prm = N.plbm_params_paper_lattice(rv, rl, xi, 2.0, 1.0, 0.8, 1.1)
    lat_ = LATTICES[lattice]
    co = syn.grid(dims)
    rho = syn.droplet(co, dims, rv, rl, R=min(dims) / 3.0, W=2.0 * xi, centre=[n / 2.0 - 0.3 for n in dims])
    f0 = syn.random_populations(lat_.Q, co, dims, 21, rho, 0.2)
    op = S.StepParams(lat_, E.PaperEOS(prm.K, prm.eos_rho_v, prm.eos_rho_l), eps=prm.epsilon, kappa=prm.kappa,
                      G=prm.G, tau_v=prm.tau_v, tau_l=prm.tau_l, rho_v=prm.rho_v, rho_l=prm.rho_l,
                      collision=collision)
    lat = Lattice(lattice, dims, prm, collision=collision, storage=storage)
    lat.write_populations(f0)
    if storage == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    steps = 4
    lat.step(steps)
    f_ref = S.run(op, f0, steps)
    tf, tu = tols(storage, steps)
    assert rel_max(lat.populations(), f_ref) <= tf
    rho_g, u = lat.moments()
    rho_r, u_r = S.moments(op, f_ref)
    assert rel_max(rho_g, rho_r) <= tf
    assert abs_max(u, u_r) <= tu
    lat.close()


@pytest.mark.parametrize("pattern", ["ab", "aa"])
def test_moments_device_equals_host_read_out(pattern):
    """plbm_moments_device writes the same float64 rho and u (SoA) into caller device buffers as
    plbm_read_moments returns on the host, at both time parities."""
    require_gpu()
    import torch
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    fmt("moments_device", pattern=pattern)
    dims = (37, 21, 13)
    lat = Lattice("D3Q19", dims, lib_params(Fg=(1e-5, 0.0, 0.0)), collision="mrt", storage="f32", pattern=pattern)
    lat.write_populations(random_state("D3Q19", dims, 31))
    for n in (3, 4):
        lat.step(n)
        rho_h, u_h = lat.moments()
        rho_d = torch.full((lat.N,), float("nan"), dtype=torch.float64, device="cuda")
        u_d = torch.full((3, lat.N), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()  # the fill runs on torch's stream, the read-out on the lattice's
        N.plbm_moments_device(lat.h, rho_d.data_ptr(), u_d.data_ptr())
        lat.stream.synchronize()
        assert np.array_equal(rho_d.cpu().numpy().reshape(rho_h.shape), rho_h)
        assert np.array_equal(u_d.cpu().numpy().reshape(u_h.shape), u_h)
    lat.close()


RESIDUAL_CASES = [c for c in CASES if c[3] == "f64"][:4] + [c for c in CASES if c[3] == "f32"][:2]


@pytest.mark.parametrize("k", [1, 7])
@pytest.mark.parametrize("case", RESIDUAL_CASES, ids=_ids)
def test_residual_matches_the_oracle(case, k):
    """The serving and convergence residual max_x |u(t) - u(t-k)| / k (u including F/2) of plbm_reduce against
    the oracle's reduce(u_prev, k).  The library keeps u(t-k) in float32: given that same rounded u(t-k), the
    oracle agrees to float64 rounding (float64 storage; float32 storage to its u bar per step); against the
    unrounded u(t-k) the difference stays within the float32 floor sqrt(d) max|u(t-k)| 2^-24 / k."""
    require_gpu()
    fmt("residual_parity", case=_ids(case), k=k)
    lattice, dims, collision, storage, walls, steps, extra = case
    lat, op, f_ref = _run_pair(*case)
    d0 = lat.reduce()
    assert d0.max_du_per_step == 0.0  # first reduction: no earlier u
    ref0, u0 = OD.reduce(op, f_ref)
    lat.step(k)
    f_k = S.run(op, f_ref, k)
    d1 = lat.reduce()
    ref_exact, _ = OD.reduce(op, f_k, u_prev=u0, dt_prev=k)
    ref_f32, u1 = OD.reduce(op, f_k, u_prev=u0.astype(np.float32).astype(np.float64), dt_prev=k)
    r = d1.max_du_per_step
    # u at both times enters; float32 storage carries its per-step u bar
    tu = 1e-13 if storage == "f64" else tols(storage, steps + k)[1]
    fmt("residual_parity_vals", lib=f"{r:.6e}", oracle=f"{ref_exact['max_du_per_step']:.6e}",
        oracle_f32_prev=f"{ref_f32['max_du_per_step']:.6e}")
    assert abs(r - ref_f32["max_du_per_step"]) <= 2 * tu / k
    floor = np.sqrt(LATTICES[lattice].d) * float(np.max(np.abs(u0))) * 2.0**-24 / k
    assert abs(r - ref_exact["max_du_per_step"]) <= floor + 2 * tu / k
    assert d1.flags == ref_exact["flags"] and d1.time == steps + k
    # the stride is the library's own time since the last reduction: 2 more steps
    lat.step(2)
    f_k2 = S.run(op, f_k, 2)
    d2 = lat.reduce()
    ref2, _ = OD.reduce(op, f_k2, u_prev=u1.astype(np.float32).astype(np.float64), dt_prev=2)
    assert abs(d2.max_du_per_step - ref2["max_du_per_step"]) <= tu
    lat.close()


def test_batch_residual_matches_the_oracle():
    """plbm_batch_diag's per-slot residual, two float64 lattices of different kinds stepped together."""
    require_gpu()
    import torch
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    fmt("batch_residual_parity")
    specs = [CASES[1], CASES[5]]
    stream = torch.cuda.Stream()
    nb = N.plbm_batch_bytes(4, 4096)
    mem = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    b = N.plbm_batch_create(4, 4096, (mem.data_ptr() + 255) // 256 * 256, nb, stream.cuda_stream)
    lats, ops, fs, slots = [], [], [], []
    for lattice, dims, collision, storage, walls, steps, extra in specs:
        f0 = random_state(lattice, dims, 9)
        op = oracle_params(lattice, collision=collision, walls=walls, **extra)
        lat = Lattice(lattice, dims, lib_params(**extra), collision=collision, storage=storage, walls=walls,
                      stream=stream)
        lat.write_populations(f0)
        lats.append(lat)
        ops.append(op)
        fs.append(f0)
        slots.append(N.plbm_batch_attach(b, lat.h))
    N.plbm_batch_diag(b, 4)  # u(0) stored
    us = [OD.reduce(op, f)[1] for op, f in zip(ops, fs)]
    k = 5
    N.plbm_batch_step(b, k)
    diag = N.plbm_batch_diag(b, 4)
    for s, op, f, u0 in zip(slots, ops, fs, us):
        ref, _ = OD.reduce(op, S.run(op, f, k), u_prev=u0.astype(np.float32).astype(np.float64), dt_prev=k)
        assert abs(diag[s].max_du_per_step - ref["max_du_per_step"]) <= 2e-13 / k
        assert diag[s].time == k and diag[s].flags == ref["flags"]
    stream.synchronize()
    N.plbm_batch_destroy(b)
    for lat in lats:
        lat.close()
