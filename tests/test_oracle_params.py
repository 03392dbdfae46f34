"""Pins of the oracle's parameter chain against what the paper fixes.

* The unit converter, K(xi) and kappa(gamma) reproduce the printed Tables II-IV
  and the five kappa values of the Young-Laplace test (Sec. VI.B).
* The paper EOS satisfies its design properties (Sec. IV): p(rho_v) = p(rho_l)
  and the Maxwell equal-area rule at exactly rho_v, rho_l.
* The general (finite psi) coexistence, width and surface tension reduce to the
  Maxwell rule and to the closed forms of Appendices A and B in the diffusive
  limit, at second order in 1/xi.
* The lattice Peng-Robinson EOS has its critical point where its constants say.
"""
import json
import os

import numpy as np
import pytest
from scipy import integrate, optimize

from oracle import eos as E
from oracle import params as P

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _fluid():
    t = GOLD["table_I_R134a_30C"]
    return P.PhysFluid(t["rho_v_kg_m3"], t["rho_l_kg_m3"], t["nu_v_mm2_s"] * 1e-6, t["nu_l_mm2_s"] * 1e-6,
                       t["gamma_mN_m"] * 1e-3)


def _close(a, printed):
    """Agreement within one unit of the last printed digit (the tables round or truncate)."""
    s = repr(float(printed))
    decimals = len(s.split(".")[1]) if "." in s and not s.endswith(".0") else 0
    return abs(a - printed) <= 10.0 ** (-decimals)


def test_table_II_planar():
    t = GOLD["table_II_planar"]
    for k, N in enumerate(t["N_x"]):
        r = P.resolve_paper(_fluid(), t["L_x_um"] * 1e-6, N, t["xi_over_dx"][k])
        assert _close(r.conv.C_L * 1e9, t["dx_nm"][k])
        assert _close(r.conv.C_T * 1e12, t["dt_ps"][k])
        assert _close(r.conv.C_U, t["C_U"][k])
        assert _close(r.conv.C_gamma, t["C_gamma"][k])


def test_table_III_droplet():
    t = GOLD["table_III_droplet"]
    for k, N in enumerate(t["N"]):
        r = P.resolve_paper(_fluid(), t["L_um"] * 1e-6, N, 1.5 * (k + 1), tau_l=t["tau_l"])
        assert _close(r.conv.C_T * 1e9, t["dt_ns"][k])
        assert _close(r.conv.C_U, t["C_U"][k])
        assert _close(r.conv.C_gamma, t["C_gamma"][k])


def test_table_IV_channel():
    t = GOLD["table_IV_channel"]
    for k, N in enumerate(t["N_y"]):
        r = P.resolve_paper(_fluid(), t["L_y_um"] * 1e-6, N, 1.5 * (k + 1), body_force=(1e6, 0, 0))
        assert _close(r.conv.C_T * 1e12, t["dt_ps"][k])
        assert _close(r.conv.C_U, t["C_U"][k])
        assert _close(r.conv.C_VF / 1e12, t["C_VF_TN_m3"][k])
        assert _close(r.conv.C_gamma, t["C_gamma"][k])
        # the body force of Sec. VI.D in lattice units is 1e6 / C_VF
        assert r.Fg[0] == pytest.approx(1e6 / r.conv.C_VF, rel=1e-15)


def test_kappa_values_young_laplace():
    g = GOLD["kappa_young_laplace"]
    for case in g["cases"]:
        r = P.resolve_paper(_fluid(), 10e-6, 100, 1.5, tau_l=case["tau_l"], gamma=case["gamma_mN_m"] * 1e-3)
        assert abs(r.kappa - case["kappa"]) <= 6e-4 * max(1.0, case["kappa"]), (case, r.kappa)


def test_fine_grid_time_step():
    f = GOLD["kappa_young_laplace"]["fine_grid"]
    r = P.resolve_paper(_fluid(), 10e-6, int(round(10.0 / f["dx_um"])), 3.0, tau_l=f["tau_l"])
    assert abs(r.conv.C_T * 1e9 - f["dt_ns"]) < 0.005


def test_liquid_density_and_viscosity_ratio():
    r = P.resolve_paper(_fluid(), 10e-6, 100, 1.5)
    d = GOLD["defaults"]
    assert r.rho_l == pytest.approx(d["rho_l_lat"], rel=1e-14)
    assert r.rho_v == pytest.approx(37.5 / 1187.0 * d["rho_l_lat"], rel=1e-14)
    # tau_v carries the vapour/liquid kinematic-viscosity ratio of Table I
    assert (r.tau_v - 0.5) / (r.tau_l - 0.5) == pytest.approx(0.339 / 0.158, rel=1e-13)


@pytest.mark.parametrize("xi", [1.5, 3.0, 7.5])
def test_paper_eos_design_properties(xi):
    rv, rl = 0.0375, 1.187
    K = P.K_from_width(xi, rv, rl)
    e = E.PaperEOS(K, rv, rl)
    p0 = e.p0()
    assert e.p(rv) == pytest.approx(p0, rel=1e-12)
    assert e.p(rl) == pytest.approx(p0, rel=1e-12)
    # Maxwell equal-area rule at exactly rho_v, rho_l (epsilon = 2 in the limit)
    val, err = integrate.quad(lambda r: (e.p(r) - p0) / r ** 2, rv, rl, epsabs=1e-16, epsrel=1e-13, limit=200)
    scale = integrate.quad(lambda r: abs(e.p(r) - p0) / r ** 2, rv, rl, limit=200)[0]
    assert abs(val) < 1e-10 * scale
    # the root finder recovers the designed coexistence
    mv, ml, mp = P.maxwell(e, rho_hi=3.0)
    assert mv == pytest.approx(rv, rel=1e-9) and ml == pytest.approx(rl, rel=1e-12)


def test_width_formula_inverts():
    rv, rl = 0.0375, 1.187
    for xi in (1.5, 3.0, 6.0):
        assert P.width_from_K(P.K_from_width(xi, rv, rl), rv, rl) == pytest.approx(xi, rel=1e-14)


def test_width_is_the_33_67_band_of_the_appendix_A_profile():
    """Appendix A profile crosses the 33 % and 67 % levels xi apart."""
    from oracle import analytic as A
    rv, rl, xi = 0.0375, 1.187, 3.0
    K = P.K_from_width(xi, rv, rl)
    r1, r2 = P.interface_levels(rv, rl)
    x1 = optimize.brentq(lambda x: A.planar_profile(np.array([x]), K, rv, rl, 0.0)[0] - r1, -50, 50, xtol=1e-13)
    x2 = optimize.brentq(lambda x: A.planar_profile(np.array([x]), K, rv, rl, 0.0)[0] - r2, -50, 50, xtol=1e-13)
    assert x2 - x1 == pytest.approx(xi, rel=1e-9)


def test_appendix_A_profile_solves_the_ode():
    """z = d sqrt(rho)/dx = -sqrt(6K)(sqrt(rho)-sqrt(rho_v))(rho-rho_l) along the profile."""
    from oracle import analytic as A
    rv, rl, xi = 0.0375, 1.187, 3.0
    K = P.K_from_width(xi, rv, rl)
    x = np.linspace(-4, 4, 81)
    h = 1e-4
    s = lambda xx: np.sqrt(A.planar_profile(xx, K, rv, rl, 0.0))
    dsdx = (s(x + h) - s(x - h)) / (2 * h)
    rho = A.planar_profile(x, K, rv, rl, 0.0)
    z = -np.sqrt(6 * K) * (np.sqrt(rho) - np.sqrt(rv)) * (rho - rl)
    assert np.max(np.abs(dsdx - z)) < 1e-7


def test_gamma_closed_form_matches_quadrature():
    """Appendix B: (kappa/9) int (d sqrt(rho)/dx)^2 dx equals the f_gamma closed form."""
    from oracle import analytic as A
    rv, rl, xi, kappa = 0.0375, 1.187, 3.0, 1.3
    K = P.K_from_width(xi, rv, rl)
    x = np.linspace(-60, 60, 240001)
    s = np.sqrt(A.planar_profile(x, K, rv, rl, 0.0))
    ds = np.gradient(s, x)
    g_quad = kappa / 9.0 * np.trapezoid(ds * ds, x)
    assert g_quad == pytest.approx(P.gamma_from_kappa(kappa, K, rv, rl), rel=1e-6)
    # and eq. (surface_tension) is its inverse
    assert P.kappa_from_gamma(g_quad, K, rv, rl) == pytest.approx(kappa, rel=1e-6)


def test_mechanical_stability_reduces_to_maxwell_in_the_limit():
    """At finite psi the eps = 2 coexistence differs from Maxwell at O(1/xi^2)."""
    rv, rl = 0.0375, 1.187
    errs = []
    for xi in (3.0, 6.0, 12.0):
        e = E.PaperEOS(P.K_from_width(xi, rv, rl), rv, rl)
        cv, cl, _ = P.coexistence(e, 2.0, rho_hi=3.0)
        errs.append(abs(cv - rv) / rv)
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.1)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.1)


def test_general_width_and_gamma_reduce_to_appendices():
    rv, rl = 0.0375, 1.187
    ew, eg = [], []
    for xi in (3.0, 6.0, 12.0):
        e = E.PaperEOS(P.K_from_width(xi, rv, rl), rv, rl)
        cv, cl, p0 = P.coexistence(e, 2.0, rho_hi=3.0)
        ew.append(abs(P.width_general(e, cv, cl, p0) - xi) / xi)
        gk = P.gamma_over_kappa_general(e, cv, cl, p0)
        eg.append(abs(gk - P.gamma_from_kappa(1.0, e.K, rv, rl)) / gk)
    for errs in (ew, eg):
        assert errs[0] > errs[1] > errs[2]
        assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.2)


def test_eps_zero_is_the_classic_shan_chen_condition():
    """eps = 0: int (p - p0) psi'/psi drho = 0, the classic mechanical-stability rule."""
    rv, rl = 0.0375, 1.187
    e = E.PaperEOS(P.K_from_width(3.0, rv, rl), rv, rl)
    cv, cl, p0 = P.coexistence(e, 0.0, rho_hi=3.0)
    # independent form of the same condition: int (p - p0) d(ln psi)
    val = integrate.quad(lambda r: (e.p(r) - p0) * (np.log(E.psi(e, r + 1e-7)) - np.log(E.psi(e, r - 1e-7))) / 2e-7,
                         cv, cl, limit=400)[0]
    assert abs(val) < 1e-9
    assert e.p(cv) == pytest.approx(p0, rel=1e-10) and e.p(cl) == pytest.approx(p0, rel=1e-10)


def test_peng_robinson_critical_point():
    """dp/drho = d2p/drho2 = 0 at T = Tc, p = pc for the lattice constants a = 2/49, b = 2/21."""
    e = E.PengRobinsonEOS(1.0)
    assert e.alpha == pytest.approx(1.0, rel=1e-15)
    h = 1e-4
    dp = lambda r: (e.p(r + h) - e.p(r - h)) / (2 * h)
    # the inflection of p at Tc: dp/drho has a minimum equal to zero
    res = optimize.minimize_scalar(dp, bounds=(0.5, 5.0), method="bounded", options={"xatol": 1e-10})
    rho_c = res.x
    # Omega_a = 0.45724 and Omega_b = 0.0778 are PR's constants rounded to 5 digits,
    # so the inflection sits at Tc to that precision
    assert abs(res.fun) < 1e-4 * e.R * e.Tc
    assert e.p(rho_c) == pytest.approx(e.pc, rel=1e-3)
    # PR's universal critical compressibility factor Z_c = pc / (rho_c R Tc) ~ 0.3074
    assert e.pc / (rho_c * e.R * e.Tc) == pytest.approx(0.3074, abs=1e-3)


def test_peng_robinson_coexistence_properties():
    e = E.PengRobinsonEOS(0.8)
    rv, rl, p0 = P.coexistence(e, 2.0)
    assert e.p(rv) == pytest.approx(p0, rel=1e-10) and e.p(rl) == pytest.approx(p0, rel=1e-10)
    assert abs(P.stability_integral(e, p0, rv, rl, 2.0)) < 1e-10
    mv, ml, mp = P.maxwell(e)
    val = integrate.quad(lambda r: (e.p(r) - mp) / r ** 2, mv, ml, limit=400)[0]
    assert abs(val) < 1e-10
    # a liquid/vapour ratio of about 30 at T/Tc = 0.8
    assert 25 < rl / rv < 40
