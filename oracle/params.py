"""Parameter chain from physical properties to lattice constants (oracle, test
infrastructure only).

* Multiphase unit converter, eqs. (unit) and (unit2), Sec. V:
      C_L = L_phs / L_lat,  C_T = C_L^2 nu_l,lat / nu_l,phs,
      C_M = C_L^3 rho_l,phs / rho_l,lat,
      C_U = C_L / C_T,  C_VF = C_M / (C_L^2 C_T^2),  C_gamma = C_M / C_T^2,
  with nu_lat = c_s^2 (tau - 1/2) (Sec. III) and r = 1 in lattice units.
* Interface width -> K = p_c / rho_c^3, eq. (thickness), Sec. IV, with f_xi of
  the same section (Appendix A derives it).
* Surface tension -> kappa, eq. (surface_tension), Sec. IV; f_gamma's rho_1 and
  rho_2 are read as rho_v and rho_l, as in Appendix B.
* Coexistence of a general EOS from the mechanical stability condition of
  Sec. IV: p(rho_v) = p(rho_l) = p_0 and
      int_{rho_v}^{rho_l} (p - p_0) psi'(rho) / psi^(1+eps) drho = 0.
* Width and surface tension of a general EOS at finite psi (lattice units,
  G = -1).  For a planar equilibrium the normal component of eq.
  (New_Pressure_Tensor) reads p_xx = p + (eps/8) psi_x^2 - (1/4) psi psi_xx = p_0,
  whose first integral is
      y(psi) = psi_x^2 = 8 psi^eps int_{psi_v}^{psi} (p - p_0) s^(-1-eps) ds,
  so x(psi) = int dpsi / sqrt(y) and gamma = int (p_xx - p_yy) dx
  = (kappa/6) int sqrt(y) dpsi.  In the diffusive limit psi -> sqrt(2 rho/3)
  these reduce to Appendices A and B.
"""
from dataclasses import dataclass

import numpy as np
from scipy import integrate, optimize

from . import eos as eosmod

CS2 = 1.0 / 3.0


# ----------------------------------------------------------------------------
# unit converter

@dataclass
class Conversion:
    C_L: float
    C_T: float
    C_M: float

    @property
    def C_U(self):
        return self.C_L / self.C_T

    @property
    def C_VF(self):
        return self.C_M / (self.C_L ** 2 * self.C_T ** 2)

    @property
    def C_gamma(self):
        return self.C_M / self.C_T ** 2

    @property
    def C_rho(self):
        return self.C_M / self.C_L ** 3

    @property
    def C_p(self):
        return self.C_M / (self.C_L * self.C_T ** 2)

    @property
    def C_nu(self):
        return self.C_L ** 2 / self.C_T


def nu_from_tau(tau):
    return CS2 * (tau - 0.5)


def tau_from_nu(nu):
    return nu / CS2 + 0.5


def converter(L_phs, L_lat, nu_l_phs, tau_l, rho_l_phs, rho_l_lat):
    C_L = L_phs / L_lat
    C_T = C_L ** 2 * nu_from_tau(tau_l) / nu_l_phs
    C_M = C_L ** 3 * rho_l_phs / rho_l_lat
    return Conversion(C_L, C_T, C_M)


# ----------------------------------------------------------------------------
# paper EOS: width and surface tension

def f_xi(rho, rho_v, rho_l):
    s, sv, sl = np.sqrt(rho), np.sqrt(rho_v), np.sqrt(rho_l)
    return (
        np.log(s - sv) / (rho_l - rho_v)
        - np.log(sl - s) / (2.0 * sl * (sl - sv))
        - np.log(s + sl) / (2.0 * sl * (sv + sl))
    )


def interface_levels(rho_v, rho_l):
    return rho_v + 0.33 * (rho_l - rho_v), rho_v + 0.67 * (rho_l - rho_v)


def K_from_width(xi, rho_v, rho_l, r=1.0):
    r1, r2 = interface_levels(rho_v, rho_l)
    return (f_xi(r1, rho_v, rho_l) - f_xi(r2, rho_v, rho_l)) ** 2 / (6.0 * r * xi ** 2)


def width_from_K(K, rho_v, rho_l, r=1.0):
    r1, r2 = interface_levels(rho_v, rho_l)
    return abs(f_xi(r1, rho_v, rho_l) - f_xi(r2, rho_v, rho_l)) / np.sqrt(6.0 * r * K)


def f_gamma(rho, rho_v, rho_l):
    sv = np.sqrt(rho_v)
    return rho ** 2 / 4.0 - rho_l * rho / 2.0 - sv * rho ** 1.5 / 3.0 + sv * rho_l * np.sqrt(rho)


def kappa_from_gamma(gamma, K, rho_v, rho_l, r=1.0):
    return np.sqrt(27.0 / (2.0 * r * K)) * gamma / (f_gamma(rho_v, rho_v, rho_l) - f_gamma(rho_l, rho_v, rho_l))


def gamma_from_kappa(kappa, K, rho_v, rho_l, r=1.0):
    """Appendix B closed form, with r placed as the derivation gives it."""
    return np.sqrt(2.0 * K / (27.0 * r)) * kappa * (f_gamma(rho_v, rho_v, rho_l) - f_gamma(rho_l, rho_v, rho_l))


# ----------------------------------------------------------------------------
# the whole chain for the paper EOS from SI inputs

@dataclass
class PhysFluid:
    rho_v: float  # kg/m^3
    rho_l: float
    nu_v: float  # m^2/s
    nu_l: float
    gamma: float  # N/m


R134A_30C = PhysFluid(rho_v=37.5, rho_l=1187.0, nu_v=0.339e-6, nu_l=0.158e-6, gamma=7.58e-3)


@dataclass
class ResolvedPaper:
    conv: Conversion
    rho_v: float
    rho_l: float
    xi: float
    K: float
    kappa: float
    gamma_lat: float
    tau_v: float
    tau_l: float
    Fg: tuple


def resolve_paper(fluid, L_phs, L_lat, xi_lat, tau_l=0.56, rho_l_lat=1.187, body_force=(0.0, 0.0, 0.0),
                  gamma=None):
    conv = converter(L_phs, L_lat, fluid.nu_l, tau_l, fluid.rho_l, rho_l_lat)
    rho_v = fluid.rho_v / conv.C_rho
    rho_l = fluid.rho_l / conv.C_rho
    K = K_from_width(xi_lat, rho_v, rho_l)
    g = fluid.gamma if gamma is None else gamma
    gamma_lat = g / conv.C_gamma
    kappa = kappa_from_gamma(gamma_lat, K, rho_v, rho_l)
    nu_v_lat = fluid.nu_v / conv.C_nu
    tau_v = tau_from_nu(nu_v_lat)
    Fg = tuple(b / conv.C_VF for b in body_force)
    return ResolvedPaper(conv, rho_v, rho_l, xi_lat, K, kappa, gamma_lat, tau_v, tau_l, Fg)


# ----------------------------------------------------------------------------
# general EOS: coexistence, width, surface tension at finite psi

def _dpsi_drho(eos, rho, h=None):
    """d psi / d rho by a central difference of psi^2 (psi' = (psi^2)' / (2 psi))."""
    rho = np.asarray(rho, dtype=np.float64)
    if h is None:
        h = 1e-6 * np.maximum(rho, 1e-3)
    r2p = eosmod.psi_radicand(eos, rho + h)
    r2m = eosmod.psi_radicand(eos, rho - h)
    return (r2p - r2m) / (2.0 * h) / (2.0 * eosmod.psi(eos, rho))


def spinodals(eos, rho_hi):
    """Local max and min of p(rho) on (0, rho_hi) (a van der Waals loop)."""
    grid = np.linspace(1e-6, rho_hi, 200001)
    p = eos.p(grid)
    dp = np.diff(p)
    sign = np.sign(dp)
    idx = np.where(np.diff(sign) != 0)[0]
    if len(idx) < 2:
        raise ValueError("EOS has no van der Waals loop below rho_hi")
    return grid[idx[0] + 1], grid[idx[1] + 1]


def _branch_roots(eos, p0, rho_max_v, rho_min_l, rho_hi):
    rv = optimize.brentq(lambda r: eos.p(r) - p0, 0.0, rho_max_v, xtol=1e-15, rtol=1e-15, maxiter=500)
    rl = optimize.brentq(lambda r: eos.p(r) - p0, rho_min_l, rho_hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    return rv, rl


def stability_integral(eos, p0, rv, rl, eps):
    def integrand(r):
        ps = eosmod.psi(eos, r)
        return (eos.p(r) - p0) * _dpsi_drho(eos, r) / ps ** (1.0 + eps)
    val, _ = integrate.quad(integrand, rv, rl, limit=400, epsabs=1e-15, epsrel=1e-12)
    return val


def _bracketed_root(g, p_lo, p_hi):
    """Root of g on (p_lo, p_hi): the highest sign change on a geometric grid, then Brent."""
    grid = np.geomspace(max(p_lo, p_hi * 1e-8) * (1 + 1e-9), p_hi * (1 - 1e-9), 25)
    # at the lowest grid pressures the vapour root sits where psi underflows to
    # zero and g is not finite; such points are skipped below
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        vals = [g(p) for p in grid]
    for k in reversed(range(len(grid) - 1)):
        if np.isfinite(vals[k]) and np.isfinite(vals[k + 1]) and vals[k] * vals[k + 1] <= 0:
            return optimize.brentq(g, grid[k], grid[k + 1], xtol=1e-16, rtol=1e-14, maxiter=500)
    raise ValueError("no coexistence pressure found in the van der Waals loop")


def coexistence(eos, eps=2.0, rho_hi=None):
    """(rho_v, rho_l, p_0) from the mechanical stability condition."""
    if rho_hi is None:
        rho_hi = 0.999 / eos.b if hasattr(eos, "b") else 10.0 * eos.rho_l
    r_max, r_min = spinodals(eos, rho_hi)
    p_hi = eos.p(r_max)
    p_lo = max(eos.p(r_min), 1e-14)

    def g(p0):
        rv, rl = _branch_roots(eos, p0, r_max, r_min, rho_hi)
        return stability_integral(eos, p0, rv, rl, eps)

    p0 = _bracketed_root(g, p_lo, p_hi)
    rv, rl = _branch_roots(eos, p0, r_max, r_min, rho_hi)
    return rv, rl, p0


def maxwell(eos, rho_hi=None):
    """Maxwell equal-area coexistence: int (p - p_0) / rho^2 drho = 0."""
    if rho_hi is None:
        rho_hi = 0.999 / eos.b if hasattr(eos, "b") else 10.0 * eos.rho_l
    r_max, r_min = spinodals(eos, rho_hi)
    p_hi = eos.p(r_max)
    p_lo = max(eos.p(r_min), 1e-14)

    def g(p0):
        rv, rl = _branch_roots(eos, p0, r_max, r_min, rho_hi)
        val, _ = integrate.quad(lambda r: (eos.p(r) - p0) / r ** 2, rv, rl, limit=400, epsabs=1e-15, epsrel=1e-12)
        return val

    p0 = _bracketed_root(g, p_lo, p_hi)
    rv, rl = _branch_roots(eos, p0, r_max, r_min, rho_hi)
    return rv, rl, p0


def _y_of_rho(eos, rho, rv, p0, eps):
    """y = psi_x^2 along the planar profile, as a function of rho."""
    def integrand(r):
        ps = eosmod.psi(eos, r)
        return (eos.p(r) - p0) * _dpsi_drho(eos, r) / ps ** (1.0 + eps)
    val, _ = integrate.quad(integrand, rv, rho, limit=400, epsabs=1e-16, epsrel=1e-12)
    return 8.0 * eosmod.psi(eos, rho) ** eps * val


def width_general(eos, rv, rl, p0, eps=2.0):
    """Distance over which rho crosses the 33 % .. 67 % band at finite psi."""
    r1, r2 = interface_levels(rv, rl)

    def integrand(r):
        y = _y_of_rho(eos, r, rv, p0, eps)
        return _dpsi_drho(eos, r) / np.sqrt(y)
    val, _ = integrate.quad(integrand, r1, r2, limit=200, epsrel=1e-10)
    return val


def gamma_over_kappa_general(eos, rv, rl, p0, eps=2.0):
    """gamma / kappa = (1/6) int sqrt(y) dpsi over the whole profile."""
    def integrand(r):
        y = max(_y_of_rho(eos, r, rv, p0, eps), 0.0)
        return np.sqrt(y) * _dpsi_drho(eos, r)
    a = rv * (1 + 1e-9)
    b = rl * (1 - 1e-9)
    val, _ = integrate.quad(integrand, a, b, limit=400, epsrel=1e-10)
    return val / 6.0
