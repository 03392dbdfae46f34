"""Pins of the oracle's lattice update against what the paper and the mathematics fix.

Each test targets a piece where a plausible mistake (a dropped term, a wrong
sign or index, a transposed operand) would show:
  * equilibrium moments (eq. Single_Phase_EDF) and Guo source moments
    (eq. Guo_Forcing_Scheme) against their defining identities;
  * M^(1), M^(2) (Sec. II) exact on quadratic fields; the Shan-Chen force of
    eq. (Shan_Chen_Force) with omega(1) = 1/3, omega(2) = 1/12 equals -G psi M^(1);
  * the interaction force sums to zero over a periodic lattice (M^(1) stencil
    antisymmetric, M^(2) symmetric);
  * streaming and half-way bounce-back move populations where they belong;
  * mass conservation, global momentum gain N F_g per step, MRT with all rates
    1/tau equal to BGK, lateral invariance and mirror symmetry;
  * the single-phase channel is Poiseuille's parabola to second order, and
    exact at the BGK half-way bounce-back magic relaxation time (2+sqrt 3)/4.
"""
import numpy as np
import pytest

import plbm_synth as syn
from oracle import eos as E
from oracle import mrt
from oracle import params as P
from oracle import step as S
from oracle.lattice import D2Q9, D3Q19

LATS = [D2Q9, D3Q19]


def _dims(lat):
    return (7, 6) if lat.d == 2 else (5, 4, 6)


def _rng_fields(lat, seed=1):
    dims = _dims(lat)
    co = syn.grid(dims)
    rho = syn.perturb(np.ones(co[0].shape) * 1.3, co, dims, seed, 0.4)
    u = syn.random_velocity(co, dims, seed, 0.08)
    F = syn.random_velocity(co, dims, seed + 1, 0.01)
    return rho, u, F


def _moment(lat, f, powers):
    out = 0.0
    for i in range(lat.Q):
        term = f[i]
        for a in powers:
            term = term * lat.c[i, a]
        out = out + term
    return out


@pytest.mark.parametrize("lat", LATS, ids=str)
def test_lattice_tables(lat):
    assert lat.w.sum() == pytest.approx(1.0, abs=4e-16)
    for a in range(lat.d):
        for b in range(lat.d):
            s = sum(lat.w[i] * lat.c[i, a] * lat.c[i, b] for i in range(lat.Q))
            assert s == pytest.approx(lat.cs2 * (a == b), abs=4e-16)
    # fourth-order isotropy: sum w c_a c_b c_g c_d = cs^4 (d_ab d_gd + d_ag d_bd + d_ad d_bg)
    for idx in np.ndindex(*(lat.d,) * 4):
        a, b, g, d = idx
        s = sum(lat.w[i] * lat.c[i, a] * lat.c[i, b] * lat.c[i, g] * lat.c[i, d] for i in range(lat.Q))
        exp = lat.cs2 ** 2 * ((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g))
        assert s == pytest.approx(exp, abs=1e-15)
    assert all(np.array_equal(lat.c[lat.opp[i]], -lat.c[i]) for i in range(lat.Q))


def test_d2q9_order_is_the_papers():
    """eq. (VelocitySet): rest, (c,0),(0,c),(-c,0),(0,-c), (c,c),(-c,c),(-c,-c),(c,-c)."""
    assert D2Q9.c.tolist() == [[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]]
    assert np.allclose(D2Q9.w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=0)


@pytest.mark.parametrize("lat", LATS, ids=str)
def test_equilibrium_moments(lat):
    rho, u, _ = _rng_fields(lat)
    feq = S.equilibrium(lat, rho, u)
    assert np.allclose(_moment(lat, feq, []), rho, rtol=1e-14, atol=0)
    for a in range(lat.d):
        assert np.allclose(_moment(lat, feq, [a]), rho * u[a], rtol=1e-13, atol=1e-16)
        for b in range(lat.d):
            exp = rho * lat.cs2 * (a == b) + rho * u[a] * u[b]
            assert np.allclose(_moment(lat, feq, [a, b]), exp, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("lat", LATS, ids=str)
def test_guo_source_moments(lat):
    rho, u, F = _rng_fields(lat)
    tau = 0.8
    src = (1 - 1 / (2 * tau)) * S.guo_source(lat, u, F)
    assert np.max(np.abs(_moment(lat, src, []))) < 1e-17
    for a in range(lat.d):
        assert np.allclose(_moment(lat, src, [a]), (1 - 1 / (2 * tau)) * F[a], rtol=1e-13, atol=1e-18)
        for b in range(lat.d):
            exp = (1 - 1 / (2 * tau)) * (F[a] * u[b] + u[a] * F[b])
            assert np.allclose(_moment(lat, src, [a, b]), exp, rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("lat", LATS, ids=str)
def test_stencil_moments_exact_on_quadratics(lat):
    """M1 = grad psi and M2 = Hessian psi exactly for a quadratic psi (interior nodes)."""
    n = 9
    dims = (n,) * lat.d
    co = [np.asarray(c, dtype=np.float64) for c in syn.grid(dims)]
    rng = np.random.default_rng(3)
    b = rng.normal(size=lat.d)
    H = rng.normal(size=(lat.d, lat.d))
    H = H + H.T
    psi = 2.0 + sum(b[a] * co[a] for a in range(lat.d))
    psi = psi + 0.5 * sum(H[a, g] * co[a] * co[g] for a in range(lat.d) for g in range(lat.d))
    M1, M2 = S.stencil_moments(lat, psi, ("periodic",) * lat.d)
    inner = (slice(1, -1),) * lat.d
    for a in range(lat.d):
        grad = b[a] + sum(H[a, g] * co[g] for g in range(lat.d))
        assert np.allclose(M1[a][inner], grad[inner], rtol=0, atol=1e-11)
        for g in range(lat.d):
            assert np.allclose(M2[a, g][inner], H[a, g], rtol=0, atol=1e-11)


def test_shan_chen_force_matches_eq_shan_chen_force():
    """eq. (Shan_Chen_Force) with omega(1) = 1/3, omega(2) = 1/12 over i = 1..8 is -G psi M1."""
    lat = D2Q9
    dims = (8, 7)
    co = syn.grid(dims)
    psi = syn.perturb(np.ones(co[0].shape), co, dims, 5, 0.5)
    G = -1.0
    omega = {1: 1 / 3, 2: 1 / 12}
    Fsc = np.zeros((2,) + psi.shape)
    for i in range(1, 9):
        pn = S.neighbour(lat, psi, lat.c[i], ("periodic", "periodic"))
        for a in range(2):
            Fsc[a] += omega[int(np.sum(lat.c[i] ** 2))] * pn * lat.c[i, a]
    Fsc = -G * psi * Fsc
    M1, M2 = S.stencil_moments(lat, psi, ("periodic", "periodic"))
    F = S.interaction_force(lat, psi, M1, M2, eps=0.0, kappa=1.0, G=G)
    assert np.allclose(F, Fsc, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("lat", LATS, ids=str)
@pytest.mark.parametrize("eps,kappa", [(2.0, 1.0), (2.0, 1.7), (0.5, 0.3)])
def test_interaction_force_sums_to_zero(lat, eps, kappa):
    dims = (9, 8) if lat.d == 2 else (6, 5, 7)
    co = syn.grid(dims)
    psi = syn.perturb(np.ones(co[0].shape), co, dims, 11, 0.6)
    M1, M2 = S.stencil_moments(lat, psi, ("periodic",) * lat.d)
    F = S.interaction_force(lat, psi, M1, M2, eps, kappa, -1.0)
    scale = np.max(np.abs(F))
    for a in range(lat.d):
        assert abs(np.sum(F[a])) < 1e-13 * scale * F[a].size
    # the corrections do matter (a dropped term would leave the SC force)
    F0 = S.interaction_force(lat, psi, M1, M2, 0.0, 1.0, -1.0)
    assert np.max(np.abs(F - F0)) > 1e-3 * scale


@pytest.mark.parametrize("lat", LATS, ids=str)
def test_streaming_moves_each_population_by_c(lat):
    dims = (5, 4) if lat.d == 2 else (5, 4, 3)
    shape = tuple(reversed(dims))
    for i in range(lat.Q):
        fpost = np.zeros((lat.Q,) + shape)
        src = (1,) * lat.d
        fpost[i][src] = 1.0
        out = S.stream(lat, fpost, ("periodic",) * lat.d)
        dst = tuple((np.array(src) + lat.c[i][::-1]) % np.array(shape))
        assert out[i][dst] == 1.0 and out.sum() == 1.0


@pytest.mark.parametrize("lat", LATS, ids=str)
def test_halfway_bounce_back(lat):
    """A population leaving the first node towards the wall returns reversed at the same node."""
    dims = (4, 5) if lat.d == 2 else (3, 4, 5)
    shape = tuple(reversed(dims))
    wall = lat.d - 1  # last component bounded
    bcs = tuple("bb" if a == wall else "periodic" for a in range(lat.d))
    for i in range(lat.Q):
        if lat.c[i, wall] != -1:
            continue
        fpost = np.zeros((lat.Q,) + shape)
        fpost[i][(0,) * lat.d] = 1.0  # node on the lower wall layer
        out = S.stream(lat, fpost, bcs)
        assert out[lat.opp[i]][(0,) * lat.d] == 1.0 and out.sum() == 1.0


_COEX = {}


def _pr_params(lat, collision="bgk", bc=None, Fg=(0.0, 0.0, 0.0), kappa=1.0, tau=1.0):
    e = E.PengRobinsonEOS(0.8)
    if "pr08" not in _COEX:
        _COEX["pr08"] = P.coexistence(e, 2.0)
    rv, rl, _ = _COEX["pr08"]
    return S.StepParams(lat, e, eps=2.0, kappa=kappa, tau_v=tau, tau_l=tau, rho_v=rv, rho_l=rl, Fg=Fg,
                        collision=collision, bc=bc), rv, rl


@pytest.mark.parametrize("lat", LATS, ids=str)
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("walls", [False, True])
def test_mass_conservation(lat, collision, walls):
    dims = (16, 12) if lat.d == 2 else (10, 9, 12)
    bc = tuple("bb" if (walls and a == lat.d - 1) else "periodic" for a in range(lat.d))
    p, rv, rl = _pr_params(lat, collision, bc)
    co = syn.grid(dims)
    rho = syn.droplet(co, dims, rv, rl, R=dims[0] / 4, W=5.0)
    f = S.init_equilibrium(lat, rho)
    m0 = np.sum(rho)
    f = S.run(p, f, 30)
    assert abs(np.sum(S.density(f)) - m0) < 1e-13 * m0


@pytest.mark.parametrize("lat", LATS, ids=str)
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_global_momentum_gain_is_body_force(lat, collision):
    dims = (14, 10) if lat.d == 2 else (8, 9, 10)
    Fg = (2e-5, -1e-5, 3e-6)[: lat.d]
    p, rv, rl = _pr_params(lat, collision, Fg=Fg)
    co = syn.grid(dims)
    rho = syn.droplet(co, dims, rv, rl, R=3.0, W=4.0, centre=[n / 2 - 0.7 for n in dims])
    f = S.init_equilibrium(lat, rho, syn.random_velocity(co, dims, 2, 0.01))
    N = rho.size
    j0 = S.first_moment(lat, f).reshape(lat.d, -1).sum(axis=1)
    steps = 10
    f = S.run(p, f, steps)
    j1 = S.first_moment(lat, f).reshape(lat.d, -1).sum(axis=1)
    for a in range(lat.d):
        assert j1[a] - j0[a] == pytest.approx(steps * N * Fg[a], rel=1e-9, abs=1e-13)


@pytest.mark.parametrize("lat", LATS, ids=str)
def test_mrt_basis_orthogonal_and_inverse(lat):
    M, Minv, classes = mrt.basis(lat)
    G = M @ M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-12)
    assert np.allclose(Minv @ M, np.eye(lat.Q), atol=1e-13)
    assert len(classes) == lat.Q


@pytest.mark.parametrize("lat", LATS, ids=str)
def test_mrt_with_all_rates_one_over_tau_is_bgk(lat):
    rho, u, F = _rng_fields(lat, 4)
    dims = _dims(lat)
    co = syn.grid(dims)
    f = syn.random_populations(lat.Q, co, dims, 9, rho)
    tau = 0.77
    feq = S.equilibrium(lat, rho, u)
    Fh = S.guo_source(lat, u, F)
    rates = {k: 1 / tau for k in ("e", "eps", "q", "m", "j", "rho", "pi")}
    a = S.collide_mrt(lat, f, feq, Fh, tau, rates)
    b = S.collide_bgk(f, feq, Fh, tau)
    assert np.max(np.abs(a - b)) < 1e-14


@pytest.mark.parametrize("lat", LATS, ids=str)
def test_mrt_conserves_mass_and_gains_force_for_any_rates(lat):
    rho, u, F = _rng_fields(lat, 6)
    dims = _dims(lat)
    co = syn.grid(dims)
    f = syn.random_populations(lat.Q, co, dims, 8, rho)
    j = S.first_moment(lat, f)
    u = (j + 0.5 * F) / S.density(f)
    rates = {"e": 0.6, "eps": 1.3, "q": 1.7, "m": 0.4, "j": 0.9, "rho": 1.1, "pi": 1.45}
    out = S.collide_mrt(lat, f, S.equilibrium(lat, S.density(f), u), S.guo_source(lat, u, F), 0.9, rates)
    assert np.allclose(S.density(out), S.density(f), rtol=1e-14)
    assert np.allclose(S.first_moment(lat, out), j + F, rtol=1e-12, atol=1e-15)


def test_mrt_shear_rate_sets_viscosity():
    """A shear wave decays at nu k^2 with nu = cs^2 (1/s_nu - 1/2), whatever the other rates.

    MRT with unrelated rates on the non-hydrodynamic moments must follow BGK
    with the same tau closely (the shear mode only sees s_nu at leading order);
    both follow exp(-nu k^2 t) up to the O(k^2) lattice correction.
    """
    lat = D2Q9
    n = 64
    dims = (1, n)
    co = syn.grid(dims)

    class Ideal:  # psi constant: no interaction force
        def p(self, rho):
            return np.asarray(rho) / 3.0 - 0.5

    tau = 0.9
    y = co[1].astype(np.float64)
    k = 2 * np.pi / n
    U = 1e-4
    u0 = np.stack([U * np.sin(k * y), np.zeros_like(y)])
    steps = 800
    amps = {}
    for coll in ("bgk", "mrt"):
        p = S.StepParams(lat, Ideal(), tau_v=tau, tau_l=tau, rho_v=0.5, rho_l=1.5, collision=coll,
                         rates={"e": 1.4, "eps": 1.2, "q": 1.6, "j": 1.0, "rho": 1.0})
        f = S.run(p, S.init_equilibrium(lat, np.ones(co[0].shape), u0), steps)
        rho, u = S.moments(p, f)
        amps[coll] = np.sum(u[0] * np.sin(k * y)) / np.sum(np.sin(k * y) ** 2) / U
    nu = lat.cs2 * (tau - 0.5)
    assert amps["mrt"] == pytest.approx(amps["bgk"], rel=2e-3)
    assert amps["bgk"] == pytest.approx(np.exp(-nu * k * k * steps), rel=5e-3)


def test_poiseuille_second_order_and_exact_at_magic_tau():
    lat = D2Q9

    class Ideal:
        def p(self, rho):
            return np.asarray(rho) / 3.0 - 0.5

    def run(tau, H, steps):
        p = S.StepParams(lat, Ideal(), tau_v=tau, tau_l=tau, rho_v=0.5, rho_l=1.5, Fg=(1e-6, 0.0),
                         bc=("periodic", "bb"))
        f = S.run(p, S.init_equilibrium(lat, np.ones((H, 1))), steps)
        rho, u = S.moments(p, f)
        y = np.arange(H) + 0.5  # walls half a spacing outside the first and last nodes
        ua = 1e-6 * y * (H - y) / (2 * lat.cs2 * (tau - 0.5))
        return np.max(np.abs(u[0, :, 0] - ua)) / ua.max(), np.max(np.abs(u[1]))

    e8, _ = run(1.0, 8, 3000)
    e16, v = run(1.0, 16, 12000)
    assert e8 / e16 == pytest.approx(4.0, rel=0.05)
    assert v < 1e-14
    em, _ = run((2 + np.sqrt(3)) / 4, 8, 4000)
    assert em < 1e-9


def test_lateral_invariance():
    """A 1-D problem on a 32 x 3 lattice equals the 32 x 1 lattice in every column."""
    lat = D2Q9
    p, rv, rl = _pr_params(lat)
    outs = []
    for ny in (1, 3):
        dims = (32, ny)
        co = syn.grid(dims)
        rho = syn.slab(co, dims, rv, rl, W=5.0, axis=0)
        outs.append(S.run(p, S.init_equilibrium(lat, rho), 20))
    for yy in range(3):
        assert np.array_equal(outs[1][:, yy, :], outs[0][:, 0, :])


@pytest.mark.parametrize("lat", LATS, ids=str)
def test_centred_droplet_is_mirror_symmetric(lat):
    dims = (16, 16) if lat.d == 2 else (10, 10, 10)
    p, rv, rl = _pr_params(lat, "mrt")
    co = syn.grid(dims)
    # nodes sit at integer positions: a centre at (n-1)/2 is mirror-symmetric
    rho = syn.droplet(co, dims, rv, rl, R=3.5, W=4.0, centre=[(n - 1) / 2 for n in dims])
    f = S.run(p, S.init_equilibrium(lat, rho), 15)
    rho, u = S.moments(p, f)
    for ax in range(lat.d):
        assert np.allclose(rho, np.flip(rho, axis=ax), rtol=1e-12)
        comp = lat.d - 1 - ax
        assert np.allclose(u[comp], -np.flip(u[comp], axis=ax), atol=1e-14)


def test_uniform_flow_is_steady():
    """A uniform density moving at constant u is an exact steady state (Galilean frame)."""
    lat = D3Q19
    p, rv, rl = _pr_params(lat, "mrt")
    dims = (6, 5, 4)
    rho = np.full(tuple(reversed(dims)), 0.9)
    u0 = np.zeros((3,) + rho.shape)
    u0[0] = 0.05
    f0 = S.init_equilibrium(lat, rho, u0)
    f = S.run(p, f0, 10)
    r, u = S.moments(p, f)
    assert np.allclose(r, 0.9, rtol=1e-14) and np.allclose(u[0], 0.05, rtol=1e-13)
