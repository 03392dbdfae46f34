"""Pins of the well-balanced oracle (oracle/wellbalanced.py) against what the
mathematics fixes, independent of its own formulas:

* the bulk chemical potential: its derivative is p'(rho)/rho (Gibbs-Duhem,
  checked by finite differences of the EOS itself), and it takes one value at
  the two coexisting densities of Maxwell's construction (the paper EOS: its
  design densities, by construction; Peng-Robinson: the equal-area densities
  of oracle.params.maxwell, computed from p alone);
* the equilibrium's moments: rho, rho u and cs^2 rho_0 I + rho u u;
* mass conservation of the update;
* the property that defines the scheme: a discrete equilibrium (a density
  field whose lattice chemical potential is uniform, found here by Newton's
  method on the lattice equations, independently of the update) at rest is
  an exact fixed point of one update: populations unchanged and u = 0 to
  round-off;
* its Laplace jump: at such an equilibrium droplet, p(rho_in) - p(rho_out)
  equals gamma / R (2-D) with gamma = int sqrt(2 k omega) d rho of the planar
  interface, to the droplet's finite-size accuracy;
* a planar equilibrium's bulk densities are the Maxwell densities.
"""
import numpy as np
import pytest
import plbm_synth as syn
from oracle import eos as E
from oracle import params as P
from oracle import step as S
from oracle import wellbalanced as W
from oracle.lattice import D2Q9, D3Q19

from wb_cases import discrete_equilibrium

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")

RV, RL = 0.0375, 1.187


def paper_eos(xi=3.0):
    return E.PaperEOS(P.K_from_width(xi, RV, RL), RV, RL)


@pytest.mark.parametrize("eos", [paper_eos(), E.PengRobinsonEOS(0.8, 0.326)], ids=["paper", "pr"])
def test_bulk_chemical_potential_follows_gibbs_duhem(eos):
    lo, hi = (0.02, 1.5) if isinstance(eos, E.PaperEOS) else (0.05, 8.0)
    r = np.linspace(lo, hi, 41)
    h = 1e-5 * r
    dmu = (W.mu_bulk(eos, r + h) - W.mu_bulk(eos, r - h)) / (2 * h)
    dp = (eos.p(r + h) - eos.p(r - h)) / (2 * h)
    assert np.max(np.abs(dmu - dp / r) / np.maximum(np.abs(dp / r), 1e-3)) < 1e-6


def test_chemical_potential_is_equal_at_maxwell_coexistence():
    e = paper_eos()
    mu = W.mu_bulk(e, np.array([RV, RL]))
    assert abs(mu[1] - mu[0]) <= 1e-14 * abs(mu[0]) + 1e-16
    pr = E.PengRobinsonEOS(0.8, 0.326)
    rv, rl, _ = P.maxwell(pr)
    mu = W.mu_bulk(pr, np.array([rv, rl]))
    assert abs(mu[1] - mu[0]) <= 1e-9 * abs(mu[0])
    # and not at the mechanical-stability densities of the pseudopotential (eps = 2)
    cv, cl, _ = P.coexistence(pr, 2.0)
    mu = W.mu_bulk(pr, np.array([cv, cl]))
    assert abs(mu[1] - mu[0]) > 1e-4


@pytest.mark.parametrize("lat", [D2Q9, D3Q19], ids=["D2Q9", "D3Q19"])
def test_equilibrium_moments(lat):
    rng = np.random.default_rng(3)
    shape = (5,) * lat.d
    rho = rng.uniform(0.04, 1.2, shape)
    u = rng.uniform(-0.08, 0.08, (lat.d,) + shape)
    rho0 = 0.0375
    feq = W.equilibrium(lat, rho, u, rho0)
    assert np.allclose(feq.sum(axis=0), rho, rtol=1e-14, atol=0)
    for a in range(lat.d):
        ja = sum(lat.c[i, a] * feq[i] for i in range(lat.Q))
        assert np.allclose(ja, rho * u[a], rtol=1e-13, atol=1e-16)
        for b in range(lat.d):
            pab = sum(lat.c[i, a] * lat.c[i, b] * feq[i] for i in range(lat.Q))
            assert np.allclose(pab, lat.cs2 * rho0 * (a == b) + rho * u[a] * u[b], rtol=1e-12, atol=1e-15)


def _wb(lat, k=0.15, tau=1.0, collision="bgk", walls=False, eos=None):
    eos = eos or paper_eos()
    bc = tuple("bb" if (walls and a == lat.d - 1) else "periodic" for a in range(lat.d))
    p = S.StepParams(lat, eos, tau_v=tau, tau_l=tau, rho_v=RV, rho_l=RL, collision=collision, bc=bc)
    return W.WBParams(p, k, RV)


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_update_conserves_mass(collision):
    wb = _wb(D2Q9, collision=collision, tau=0.8)
    dims = (24, 20)
    co = syn.grid(dims)
    rho = syn.droplet(co, dims, RV, RL, R=6.0, W=6.0)
    f = syn.random_populations(9, co, dims, 5, rho, 0.1)
    m0 = f.sum()
    f = W.run(wb, f, 20)
    assert abs(f.sum() - m0) <= 1e-13 * m0


@pytest.fixture(scope="module")
def droplet_equilibrium():
    dims = (128, 128)
    k = 0.15
    e = paper_eos()
    co = syn.grid(dims)
    rho = discrete_equilibrium(e, k, syn.droplet(co, dims, RV, RL, R=32.0, W=6.0))
    return dims, k, e, rho


def test_discrete_equilibrium_is_a_fixed_point(droplet_equilibrium):
    dims, k, e, rho = droplet_equilibrium
    wb = _wb(D2Q9, k=k, eos=e)
    mu = W.chemical_potential(wb, rho)
    assert np.ptp(mu) <= 1e-13 * np.max(np.abs(mu))  # the solve reached a uniform chemical potential
    assert rho.max() > 0.9 * RL and rho.min() < 2 * RV  # a droplet, not the uniform state
    f0 = W.init_equilibrium(wb, rho)
    r0, u0 = W.moments(wb, f0)
    assert np.max(np.abs(u0)) <= 1e-15
    f1 = W.step(wb, f0)
    assert np.max(np.abs(f1 - f0)) <= 1e-14 * np.max(np.abs(f0))
    _, u1 = W.moments(wb, f1)
    assert np.max(np.abs(u1)) <= 1e-15
    # with MRT, and across a few steps, too
    wbm = _wb(D2Q9, k=k, eos=e, collision="mrt")
    f5 = W.run(wbm, f0, 5)
    assert np.max(np.abs(f5 - f0)) <= 1e-13 * np.max(np.abs(f0))


def test_pseudopotential_force_is_not_balanced_at_that_state(droplet_equilibrium):
    """The same density field at rest under the paper's discretisation carries a velocity (F/2 rho) of the
    size of its spurious currents: the balance above is specific to the well-balanced form."""
    dims, k, e, rho = droplet_equilibrium
    p = S.StepParams(D2Q9, e, tau_v=1.0, tau_l=1.0, rho_v=RV, rho_l=RL)
    _, u = S.moments(p, S.init_equilibrium(D2Q9, rho))
    assert np.max(np.abs(u)) > 1e-4


def test_equilibrium_droplet_obeys_young_laplace(droplet_equilibrium):
    dims, k, e, rho = droplet_equilibrium
    r_in, r_out = rho[64, 64], rho[0, 0]
    frac = np.sum((rho - r_out) / (r_in - r_out))
    R_eq = np.sqrt(frac / np.pi)
    dp = e.p(r_in) - e.p(r_out)
    gamma = W.gamma_planar(e, k, RV, RL)
    # measured 0.9994 of gamma at R_eq = 31.7 (0.9993 at 63.6): bar 1 %
    assert dp * R_eq == pytest.approx(gamma, rel=0.01)


def test_planar_equilibrium_has_the_maxwell_densities():
    e = paper_eos()
    k = 0.15
    dims = (1, 160)
    co = syn.grid(dims)
    rho = discrete_equilibrium(e, k, syn.slab(co, dims, RV, RL, W=6.0, axis=1))
    assert rho.max() == pytest.approx(RL, rel=1e-4)
    assert rho.min() == pytest.approx(RV, rel=1e-3)
