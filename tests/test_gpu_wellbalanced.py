"""The well-balanced scheme on the GPU (descriptor scheme = PLBM_SCHEME_WELL_BALANCED).

1. One to four updates of random non-equilibrium states against the oracle's
   well-balanced update (oracle/wellbalanced.py), D2Q9 and D3Q19, BGK and MRT,
   periodic and walled, float64 (bar 1e-12) and float32 (gpu_cases.tols);
   moments and reductions too.
2. A discrete equilibrium droplet (uniform lattice chemical potential, found on
   the host by Newton's method from the oracle's equations) is a fixed point on
   the GPU: 1000 float64 updates leave populations and u = 0 unchanged to
   round-off.
3. A static droplet started from a tanh profile: its spurious currents decay
   to round-off under the well-balanced scheme (float64), while the paper's
   discretisation of the same fluid keeps them; the settled droplet obeys
   Young-Laplace with the scheme's planar surface tension.
4. In a batch beside a pseudopotential lattice, a well-balanced lattice steps
   bitwise as it does alone.
5. Periodic marching axes of one to three planes (shorter than the planes
   both launches load ahead) wrap inside an exact-size buffer.
6. The benchmark's 256^3 workload, float32 and float64: sampled windows
   against the oracle on light-cone-padded boxes.
The fluid is the paper's EOS (R134a-like lattice densities 0.0375 / 1.187,
interface width parameter xi = 3), gradient coefficient k = 0.15.
"""
import numpy as np
import pytest

import plbm_synth as syn
from oracle import eos as E
from oracle import params as P
from oracle import step as S
from oracle import wellbalanced as W
from oracle.lattice import LATTICES

from gpu_cases import abs_max, fmt, rel_max, require_gpu, tols

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")]

RV, RL, XI, K_GRAD = 0.0375, 1.187, 3.0, 0.15


def _oracle(lattice, collision, walls, tau_v, tau_l, Fg=(0.0, 0.0, 0.0)):
    lat = LATTICES[lattice]
    e = E.PaperEOS(P.K_from_width(XI, RV, RL), RV, RL)
    cv, cl, _ = P.coexistence(e, 2.0)  # tau(rho) anchors, as the library resolves them
    bc = tuple("bb" if (walls and a == lat.d - 1) else "periodic" for a in range(lat.d))
    p = S.StepParams(lat, e, tau_v=tau_v, tau_l=tau_l, rho_v=cv, rho_l=cl, collision=collision, bc=bc,
                     Fg=tuple(Fg[: lat.d]) + (0.0,) * (3 - lat.d))
    return W.WBParams(p, K_GRAD, RV)


def _lattice(lattice, dims, collision, storage, walls, tau_v, tau_l, Fg=(0.0, 0.0, 0.0)):
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    prm = N.plbm_params_paper_lattice(RV, RL, XI, 2.0, 1.0, tau_v, tau_l, list(Fg))
    return Lattice(lattice, dims, prm, collision=collision, storage=storage, walls=walls, wb_k=K_GRAD, wb_rho0=RV)


CASES = [
    # lattice, dims, collision, storage, walls, steps, tau_v, tau_l, Fg
    ("D2Q9", (37, 29), "bgk", "f64", False, 4, 1.0, 1.0, (0.0, 0.0, 0.0)),
    ("D2Q9", (40, 33), "mrt", "f64", True, 4, 0.8, 1.1, (1e-5, 0.0, 0.0)),
    ("D3Q19", (21, 17, 13), "mrt", "f64", False, 3, 0.9, 1.2, (0.0, 0.0, 0.0)),
    ("D3Q19", (20, 16, 12), "bgk", "f64", True, 3, 1.0, 1.0, (2e-6, -1e-6, 0.0)),
    ("D3Q19", (35, 17, 10), "mrt", "f32", False, 3, 1.0, 1.0, (0.0, 0.0, 0.0)),
    ("D2Q9", (70, 37), "bgk", "f32", True, 4, 0.8, 1.1, (0.0, 0.0, 0.0)),
]


def _ids(c):
    return f"{c[0]}-{'x'.join(map(str, c[1]))}-{c[2]}-{c[3]}-{'bb' if c[4] else 'per'}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_wb_step_matches_the_oracle(case):
    require_gpu()
    lattice, dims, collision, storage, walls, steps, tau_v, tau_l, Fg = case
    fmt("wb_parity", case=_ids(case))
    wb = _oracle(lattice, collision, walls, tau_v, tau_l, Fg)
    lat = _lattice(lattice, dims, collision, storage, walls, tau_v, tau_l, Fg)
    co = syn.grid(dims)
    rho = syn.droplet(co, dims, RV, RL, R=min(dims) / 3.0, W=2 * XI, centre=[n / 2.0 - 0.3 for n in dims])
    f0 = syn.random_populations(LATTICES[lattice].Q, co, dims, 11, rho, 0.2)
    lat.write_populations(f0)
    if storage == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    d0 = lat.reduce()
    lat.step(steps)
    ref = W.run(wb, f0, steps)
    tf, tu = tols(storage, steps)
    f = lat.populations()
    rho_g, u_g = lat.moments()
    rho_r, u_r = W.moments(wb, ref)
    fmt("wb_parity_err", rel_f=f"{rel_max(f, ref):.2e}", rel_rho=f"{rel_max(rho_g, rho_r):.2e}",
        abs_u=f"{abs_max(u_g, u_r):.2e}")
    assert rel_max(f, ref) <= tf
    assert rel_max(rho_g, rho_r) <= tf
    assert abs_max(u_g, u_r) <= tu
    d = lat.reduce()
    assert d.mass == pytest.approx(float(np.sum(rho_r)), rel=1e-12 if storage == "f64" else 1e-6)
    assert d.max_u == pytest.approx(float(np.max(np.sqrt((u_r ** 2).sum(axis=0)))), rel=1e-9, abs=tu)
    # mass is conserved by the update
    assert d.mass == pytest.approx(d0.mass, rel=1e-13 if storage == "f64" else 1e-6)
    assert d.flags == 0 and d.time == steps
    lat.close()


def _newton_droplet(n, R):
    from wb_cases import discrete_equilibrium
    e = E.PaperEOS(P.K_from_width(XI, RV, RL), RV, RL)
    co = syn.grid((n, n))
    return discrete_equilibrium(e, K_GRAD, syn.droplet(co, (n, n), RV, RL, R=R, W=2 * XI))


def test_discrete_equilibrium_is_a_fixed_point_on_the_gpu():
    require_gpu()
    fmt("wb_fixed_point")
    n = 128
    rho = _newton_droplet(n, 32.0)
    for collision in ("bgk", "mrt"):
        lat = _lattice("D2Q9", (n, n), collision, "f64", False, 0.8, 1.1)
        lat.init_fields(rho)
        f0 = lat.populations()
        lat.step(1000)
        f1 = lat.populations()
        _, u = lat.moments()
        fmt("wb_fixed_point_err", collision=collision, rel_f=f"{rel_max(f1, f0):.2e}", max_u=f"{np.abs(u).max():.2e}")
        assert rel_max(f1, f0) <= 1e-13
        assert np.abs(u).max() <= 1e-14
        lat.close()


def test_spurious_currents_fall_to_round_off_and_laplace_holds():
    require_gpu()
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    fmt("wb_static_droplet")
    n, R = 128, 32.0
    e = E.PaperEOS(P.K_from_width(XI, RV, RL), RV, RL)
    lat = _lattice("D2Q9", (n, n), "bgk", "f64", False, 1.0, 1.0)
    lat.init_shape(N.PLBM_SHAPE_DROPLET, RL, RV, W=2 * XI, R=R)
    history = []
    for _ in range(40):
        lat.step(50_000)
        d = lat.reduce()
        history.append(d.max_u)
        if d.max_u < 1e-14:
            break
    fmt("wb_static_droplet_max_u", history=" ".join(f"{v:.1e}" for v in history))
    assert history[-1] <= 1e-13
    rho, u = lat.moments()
    lat.close()
    r_in, r_out = rho[n // 2, n // 2], rho[0, 0]
    R_eq = np.sqrt(np.sum((rho - r_out) / (r_in - r_out)) / np.pi)
    gamma = W.gamma_planar(e, K_GRAD, RV, RL)
    dpR = (e.p(r_in) - e.p(r_out)) * R_eq
    fmt("wb_laplace", R_eq=f"{R_eq:.3f}", dpR_over_gamma=f"{dpR / gamma:.5f}")
    assert dpR == pytest.approx(gamma, rel=0.01)
    # the paper's discretisation of the same fluid and droplet keeps spurious currents
    prm = N.plbm_params_paper_lattice(RV, RL, XI, 2.0, 1.0, 1.0, 1.0, [0.0, 0.0, 0.0])
    pp = Lattice("D2Q9", (n, n), prm, collision="bgk", storage="f64")
    pp.init_shape(N.PLBM_SHAPE_DROPLET, RL, RV, W=2 * XI, R=R)
    pp.step(200_000)
    d = pp.reduce()
    fmt("pseudopotential_static_droplet", max_u=f"{d.max_u:.2e}")
    assert d.max_u > 1e-6
    pp.close()


def test_wb_lattices_step_in_a_batch_like_alone():
    """A well-balanced lattice and a pseudopotential one share a batch (separate launch groups, the
    well-balanced group two launches per step): after batched steps, each lattice's populations and
    reduction equal those of its solo twin, bitwise."""
    require_gpu()
    import torch
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    from gpu_cases import lib_params
    fmt("wb_batched")
    prm = N.plbm_params_paper_lattice(RV, RL, XI, 2.0, 1.0, 0.9, 1.1, [0.0, 0.0, 0.0])
    stream = torch.cuda.Stream()
    made = []

    def make(kind, dims, params, **kw):
        pair = []
        for s in (stream, None):
            lat = Lattice(kind, dims, params, collision="mrt", storage="f32", stream=s, **kw)
            lat.init_shape(N.PLBM_SHAPE_DROPLET, params.rho_l, params.rho_v, W=6.0, R=min(dims) / 4.0)
            pair.append(lat)
        made.extend(pair)
        return pair

    wb_b, wb_s = make("D3Q19", (37, 21, 15), prm, wb_k=K_GRAD, wb_rho0=RV)
    pp_b, pp_s = make("D2Q9", (70, 41), lib_params())
    nb = N.plbm_batch_bytes(4, 4096)
    mem = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    b = N.plbm_batch_create(4, 4096, (mem.data_ptr() + 255) // 256 * 256, nb, stream.cuda_stream)
    for lat in (wb_b, pp_b):
        lat.reduce()
        N.plbm_batch_attach(b, lat.h)
    N.plbm_batch_step(b, 37)
    diag = N.plbm_batch_diag(b, 4)
    stream.synchronize()
    for solo in (wb_s, pp_s):
        solo.reduce()
        solo.step(37)
    d_solo = [wb_s.reduce(), pp_s.reduce()]
    for k, (bat, solo) in enumerate(((wb_b, wb_s), (pp_b, pp_s))):
        assert np.array_equal(bat.populations(), solo.populations()), k
        assert diag[k].mass == d_solo[k].mass and diag[k].max_u == d_solo[k].max_u, k
        assert diag[k].flags == 0 and diag[k].time == 37
    N.plbm_batch_destroy(b)
    for lat in made:
        lat.close()

SHORT_AXES = [
    # lattice, dims (the last axis is the kernel's marching axis), steps
    ("D3Q19", (5, 3, 1), 3),
    ("D3Q19", (5, 3, 2), 3),
    ("D3Q19", (4, 3, 3), 4),
    ("D2Q9", (7, 1), 3),
    ("D2Q9", (7, 2), 4),
]


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", SHORT_AXES, ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[1]))}")
def test_wb_short_periodic_marching_axis_stays_inside_the_lattice(case, storage):
    """Both launches of a well-balanced step load planes ahead of their use (the
    chemical-potential pass three planes of populations, the update its mu
    ring); a periodic marching axis shorter than that window must wrap inside
    the lattice's arrays.  The lattice sits at the start of a buffer whose
    remaining megabyte holds all-ones bytes (NaN in float32 and float64): a read
    past the lattice would carry a NaN into the state (the reduction's NaN flag,
    and parity); the bytes after the lattice stay untouched."""
    require_gpu()
    import torch
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import make_desc

    lattice, dims, steps = case
    fmt("wb_short_axis", case=case, storage=storage)
    wb = _oracle(lattice, "mrt", False, 0.9, 1.1)
    prm = N.plbm_params_paper_lattice(RV, RL, XI, 2.0, 1.0, 0.9, 1.1, [0.0, 0.0, 0.0])
    desc = make_desc(lattice, dims, "mrt", storage, wb_k=K_GRAD, wb_rho0=RV)
    nb = N.plbm_lattice_bytes(desc)
    mem = torch.full((nb + 256 + (1 << 20),), 0xFF, dtype=torch.uint8, device="cuda")
    ptr = (mem.data_ptr() + 255) // 256 * 256
    stream = torch.cuda.Stream()
    h = N.plbm_create(desc, prm, ptr, nb, stream.cuda_stream)
    Q = LATTICES[lattice].Q
    try:
        co = syn.grid(dims)
        rho = syn.droplet(co, dims, RV, RL, R=1.2, W=2.0, centre=[n / 2.0 for n in dims])
        f_in = syn.random_populations(Q, co, dims, 41, rho, 0.05)
        N.plbm_write_populations(h, f_in.reshape(-1))
        ref = f_in if storage == "f64" else f_in.astype(np.float32).astype(np.float64)
        for _ in range(steps):
            d = N.plbm_reduce(h, True)
            assert d.flags == 0, d.flags
            N.plbm_step(h, 1)
        d = N.plbm_reduce(h, True)
        assert d.flags == 0, d.flags
        ref = W.run(wb, ref, steps)
        f = N.plbm_read_populations(h, Q, int(np.prod(dims))).reshape(ref.shape)
        tf, _ = tols(storage, steps)
        err = rel_max(f, ref)
        fmt("wb_short_axis_err", err=f"{err:.3e}", tol=f"{tf:.3e}")
        assert err <= tf
        stream.synchronize()
        assert bool((mem[ptr - mem.data_ptr() + nb:] == 0xFF).all())
    finally:
        stream.synchronize()
        N.plbm_destroy(h)


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_wb_droplet_256cubed_mrt_windows(storage):
    """The benchmark's well-balanced workload at full size: D3Q19 256^3, MRT, the paper's EOS with k = 0.15,
    droplet R = 48 (tanh width 2 xi), stepped 8 times through the replay graphs.  The update at a node reads
    populations one node away, the chemical potential one node further and the density one beyond that, so
    after K steps a node depends on the initial state within 3K nodes, and its moments (the force's chemical
    potential) within 3K + 2: windows of 8^3 nodes (interface, centre, a corner wrapped across three faces,
    vapour) must match the oracle run on periodic boxes with a 3K + 2 margin."""
    require_gpu()
    fmt("wb_fullsize", storage=storage)
    dims, steps, out = (256, 256, 256), 8, 8
    wb = _oracle("D3Q19", "mrt", False, 1.0, 1.0)
    lat = _lattice("D3Q19", dims, "mrt", storage, False, 1.0, 1.0)

    def rho_fn(co):
        return syn.droplet(co, dims, RV, RL, R=48.0, W=2 * XI)

    lat.init_fields(rho_fn(syn.grid(dims)))
    lat.step(steps)
    f_gpu = lat.populations()
    _, u_gpu = lat.moments()
    d = lat.reduce()
    lat.close()
    assert d.flags == 0 and d.time == steps
    m = 3 * steps + 2
    tf, tu = tols(storage, steps)
    bad = []
    for lo in [(172, 124, 124), (124, 124, 124), (252, 250, 251), (100, 170, 30)]:
        co = syn.window(dims, [a - m for a in lo], [out + 2 * m] * 3)
        f0 = W.init_equilibrium(wb, rho_fn(co))
        if storage == "f32":
            f0 = f0.astype(np.float32).astype(np.float64)
        # the box is periodic on the oracle's side only: its seams lie outside the interior's light cone
        with np.errstate(over="ignore", invalid="ignore"):
            ref = W.run(wb, f0, steps)
            rho_r, u_r = W.moments(wb, ref)
        inner = tuple(slice(m, m + out) for _ in range(3))
        idx = np.ix_(*[(np.arange(out) + lo[a]) % dims[a] for a in (2, 1, 0)])
        got = f_gpu[(slice(None),) + idx]
        err = rel_max(got, ref[(slice(None),) + inner])
        dev = np.abs(got - ref[(slice(None),) + inner])
        at = np.unravel_index(int(np.argmax(dev)), dev.shape)
        fmt("wb_window", lo=lo, rel_f=f"{err:.3e}", tol=f"{tf:.1e}", worst=at, f=f"{float(ref[(slice(None),) + inner][at]):.6e}",
            rho=f"{float(rho_r[inner][at[1:]]):.6e}", u=f"{abs_max(u_gpu[(slice(None),) + idx], u_r[(slice(None),) + inner]):.2e}")
        bad += [(lo, "f", err)] if err > tf else []
        e_rho = rel_max(got.sum(axis=0), rho_r[inner])
        bad += [(lo, "rho", e_rho)] if e_rho > tf else []
        e_u = abs_max(u_gpu[(slice(None),) + idx], u_r[(slice(None),) + inner])
        bad += [(lo, "u", e_u)] if e_u > tu else []
    assert not bad, bad

