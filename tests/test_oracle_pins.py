"""Pins of three oracle functions against what physics and mathematics fix,
independent of the functions' own formulas.  Each test also plants a
plausible mistake in the oracle (on the CPU, through monkeypatch) and checks
that the pin catches it.

* Peng-Robinson temperature function alpha(T_r, omega) (an extension; the
  paper uses its own EOS): the acentric factor is defined by the reduced
  saturation pressure at T_r = 0.7, omega = -log10(p_sat / p_c) - 1, so the
  EOS's own Maxwell coexistence pressure there must return the omega it was
  built with.  Away from 0.7: sqrt(alpha) is linear in sqrt(T_r) (its
  derivative in sqrt(T_r) is one constant, -m(omega)), alpha(1) = 1, and the
  saturation pressure follows the Edmister two-point vapour-pressure relation
  log10(p_sat / p_c) = 7/3 (1 + omega)(1 - 1/T_r) between T_r = 0.7 and 1.
* Density-weighted relaxation time tau(rho) (Sec. VI, linear between tau_v at
  rho_v and tau_l at rho_l; nu = c_s^2 (tau - 1/2), Sec. III): a small shear
  wave in a uniform fluid at rho_v, the mid density and rho_l, stepped by the
  full oracle update, decays at nu(tau(rho)) k^2.
* Two-phase channel reference (Sec. VI.D; the paper prints no formula): for a
  constant viscosity it must be the Poiseuille parabola, for a sharp two-layer
  density the piecewise closed form of two Newtonian layers with continuous
  velocity and shear stress.
"""
import numpy as np
import pytest

from oracle import analytic as A
from oracle import eos as E
from oracle import params as P
from oracle import step as S
from oracle.lattice import D2Q9

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


def _omega_recovered(omega):
    e = E.PengRobinsonEOS(0.7, omega)
    _, _, p_sat = P.maxwell(e)
    return -np.log10(p_sat / e.pc) - 1.0


@pytest.mark.parametrize("omega", [0.0, 0.326, 0.5])
def test_pr_alpha_reproduces_the_acentric_factor_definition(omega):
    # Peng and Robinson fitted m(omega) to vapour pressures, so the definition holds to a few 1e-3
    assert abs(_omega_recovered(omega) - omega) <= 5e-3


def test_pr_acentric_pin_catches_a_wrong_m_coefficient(monkeypatch):
    c = E.PR_OMEGA_COEF
    monkeypatch.setattr(E, "PR_OMEGA_COEF", (c[0], c[1], -c[2]))  # sign of the omega^2 term
    assert abs(_omega_recovered(0.326) - 0.326) > 5e-3
    monkeypatch.setattr(E, "PR_OMEGA_COEF", (c[0], 1.45226, c[2]))  # a digit of the omega term
    assert abs(_omega_recovered(0.326) - 0.326) > 5e-3


def _edmister_ratio(tr, omega=0.326):
    e = E.PengRobinsonEOS(tr, omega)
    _, _, p_sat = P.maxwell(e)
    return (p_sat / e.pc) / 10.0 ** (7.0 / 3.0 * (1.0 + omega) * (1.0 - 1.0 / tr))


def test_pr_alpha_temperature_dependence():
    omega = 0.326
    assert E.PengRobinsonEOS(1.0, omega).alpha == 1.0
    trs = np.array([0.55, 0.7, 0.85, 1.0, 1.2])
    sa = np.array([np.sqrt(E.PengRobinsonEOS(t, omega).alpha) for t in trs])
    slopes = np.diff(sa) / np.diff(np.sqrt(trs))
    assert np.ptp(slopes) <= 1e-12 * abs(slopes[0])
    # the same constant slope for another omega, steeper for a larger acentric factor
    sa2 = [np.sqrt(E.PengRobinsonEOS(t, 0.5).alpha) for t in (0.6, 0.9)]
    assert (sa2[1] - sa2[0]) / (np.sqrt(0.9) - np.sqrt(0.6)) < slopes[0] < 0
    for tr in (0.8, 0.9):
        assert abs(_edmister_ratio(tr) - 1.0) <= 0.02


def test_pr_temperature_pin_catches_a_wrong_temperature_form(monkeypatch):
    def alpha_linear_in_tr(self):  # T_r where sqrt(T_r) belongs
        c = E.PR_OMEGA_COEF
        m = c[0] + c[1] * self.omega + c[2] * self.omega ** 2
        return (1.0 + m * (1.0 - self.T_over_Tc)) ** 2

    monkeypatch.setattr(E.PengRobinsonEOS, "alpha", property(alpha_linear_in_tr))
    assert abs(_edmister_ratio(0.8) - 1.0) > 0.02


# ---- tau(rho): viscosity measured from shear-wave decay ----

def _shear_wave_nu(p, rho0, ny=64, amp=1e-6, t1=100, t2=400):
    """Kinematic viscosity from the decay of u_x = amp sin(k y) in a uniform fluid of density rho0."""
    dims = (1, ny)
    y = np.arange(ny, dtype=np.float64).reshape(ny, 1)
    k = 2.0 * np.pi / ny
    rho = np.full((ny, 1), rho0)
    u = np.zeros((2, ny, 1))
    u[0] = amp * np.sin(k * y)
    f = S.init_equilibrium(D2Q9, rho, u)
    s = np.sin(k * y)

    def amplitude(f):
        _, uu = S.moments(p, f)
        return 2.0 / ny * float(np.sum(uu[0] * s))

    f = S.run(p, f, t1)
    a1 = amplitude(f)
    f = S.run(p, f, t2 - t1)
    a2 = amplitude(f)
    assert dims == (1, ny)
    return np.log(a1 / a2) / (k * k * (t2 - t1))


def _pr_params(collision, tau_v=0.6, tau_l=1.3):
    e = E.PengRobinsonEOS(0.8, 0.326)
    rv, rl, _ = P.coexistence(e, 2.0)
    return S.StepParams(D2Q9, e, eps=2.0, kappa=1.0, tau_v=tau_v, tau_l=tau_l, rho_v=rv, rho_l=rl,
                        collision=collision)


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_tau_of_rho_from_shear_wave_decay(collision):
    p = _pr_params(collision)
    rv, rl = p.rho_v, p.rho_l
    cs2 = 1.0 / 3.0
    # expected: tau_v at rho_v, tau_l at rho_l, their mean at the mean density
    for rho0, tau in ((rv, p.tau_v), (0.5 * (rv + rl), 0.5 * (p.tau_v + p.tau_l)), (rl, p.tau_l)):
        nu = _shear_wave_nu(p, rho0)
        assert nu == pytest.approx(cs2 * (tau - 0.5), rel=5e-3), (collision, rho0, nu)


def test_tau_pin_catches_swapped_phases(monkeypatch):
    p = _pr_params("bgk")
    monkeypatch.setattr(S, "tau_of_rho", lambda p, rho: p.tau_l + (rho - p.rho_v) / (p.rho_l - p.rho_v)
                        * (p.tau_v - p.tau_l))
    nu = _shear_wave_nu(p, p.rho_v)
    assert abs(nu / ((p.tau_v - 0.5) / 3.0) - 1.0) > 5e-3


# ---- the channel reference ----

def _two_layer(y, F, mu1, mu2, h, H):
    """u(y) of two Newtonian layers (mu1 below y = h, mu2 above) between no-slip walls at 0 and H under a
    uniform body force F: mu u' = C - F y in each layer, u continuous, u(0) = u(H) = 0."""
    # u(H) = (C h - F h^2/2)/mu1 + (C (H - h) - F (H^2 - h^2)/2)/mu2 = 0
    C = F * (h * h / (2 * mu1) + (H * H - h * h) / (2 * mu2)) / (h / mu1 + (H - h) / mu2)
    y = np.asarray(y, dtype=np.float64)
    lower = (C * y - F * y * y / 2) / mu1
    upper = (C * h - F * h * h / 2) / mu1 + (C * (y - h) - F * (y * y - h * h) / 2) / mu2
    return np.where(y <= h, lower, upper)


def test_channel_velocity_is_poiseuille_for_constant_viscosity():
    H, F, rho, nu = 64.0, 1e-6, 1.7, 0.11
    y = np.linspace(0.0, H, 33)
    u = A.channel_velocity(y, lambda s: np.full_like(s, rho), lambda r: np.full_like(r, nu), F, H)
    mu = rho * nu
    ref = F * y * (H - y) / (2.0 * mu)
    assert np.max(np.abs(u - ref)) <= 1e-9 * np.max(ref)


def test_channel_velocity_is_the_two_layer_closed_form_for_a_step_density():
    H, F, h = 128.0, 1e-6, 64.0
    rv, rl, nu_v, nu_l = 0.25, 7.19, 0.21, 0.07  # liquid below the interface
    y = np.linspace(0.0, H, 129)

    def rho_of_y(s):
        return np.where(s < h, rl, rv)

    def nu_of_rho(r):
        return np.where(r > 0.5 * (rv + rl), nu_l, nu_v)

    u = A.channel_velocity(y, rho_of_y, nu_of_rho, F, H)
    ref = _two_layer(y, F, rl * nu_l, rv * nu_v, h, H)
    # the trapezoid straddles the viscosity jump once: an error of half a quadrature step
    assert np.max(np.abs(u - ref)) <= 1e-4 * np.max(np.abs(ref))
    # the faster vapour layer: the maximum lies above the interface
    assert y[np.argmax(u)] > h


def test_channel_pin_catches_a_dropped_reciprocal(monkeypatch):
    H, F, h = 128.0, 1e-6, 64.0
    rv, rl, nu_v, nu_l = 0.25, 7.19, 0.21, 0.07
    y = np.linspace(0.0, H, 129)
    orig = A.channel_velocity

    def mu_instead_of_inverse(y, rho_of_y, nu_of_rho, F, H, n_quad=20001):
        # the integrands use mu where 1/mu belongs
        return orig(y, lambda s: 1.0 / rho_of_y(s), lambda r: 1.0 / nu_of_rho(1.0 / r), F, H, n_quad)

    monkeypatch.setattr(A, "channel_velocity", mu_instead_of_inverse)
    u = A.channel_velocity(y, lambda s: np.where(s < h, rl, rv),
                           lambda r: np.where(r > 0.5 * (rv + rl), nu_l, nu_v), F, H)
    ref = _two_layer(y, F, rl * nu_l, rv * nu_v, h, H)
    assert np.max(np.abs(u - ref)) > 1e-4 * np.max(np.abs(ref))
