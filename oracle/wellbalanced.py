"""Well-balanced discretisation of the two-phase update (oracle, test
infrastructure only).

Sec. VI.B of the paper notes that its discretisation keeps spurious currents
at a static droplet and points to well-balanced schemes (its reference to
Guo's well-balanced lattice Boltzmann model) as the way to remove them.  The
paper states none of that scheme's equations; this module is the reading
taken here, built on the property that defines a well-balanced scheme: a
discrete mechanical equilibrium (fluid at rest, chemical potential uniform on
the lattice) is an exact steady state of the discrete update, so the velocity
at equilibrium is zero to round-off.  Two changes to the update give it:

* the force is written in potential form, F = -rho grad_d mu + F_g, with the
  lattice chemical potential
      mu(x) = mu_b(rho(x)) - k lap_d rho(x),
  mu_b the bulk chemical potential of the same equation of state
  (d mu_b / d rho = p'(rho) / rho, Gibbs-Duhem), k a gradient coefficient
  that sets the interface width and the surface tension, and the isotropic
  lattice operators
      grad_d g(x) = sum_i w_i c_i g(x + c_i) / cs^2,
      lap_d  g(x) = 2 sum_i w_i (g(x + c_i) - g(x)) / cs^2;
  a uniform mu makes F vanish exactly, whatever the density field;
* the equilibrium carries a constant reference density rho_0 on the moving
  populations at rest,
      f_i^eq = w_i rho_0 + delta_i0 (rho - rho_0) + w_i rho s_i(u),
      s_i(u) = c_i.u / cs^2 + (c_i.u)^2 / (2 cs^4) - u.u / (2 cs^2),
  so its moments are rho, rho u and cs^2 rho_0 I + rho u u: at rest the
  streamed populations are uniform and streaming leaves them unchanged, and
  the whole pressure comes from the force (Gibbs-Duhem: rho grad mu = grad p
  in the bulk).

Everything else is the update of ``oracle.step``: u = (sum f c + F/2)/rho,
tau(rho), BGK or MRT collision with Guo forcing, streaming with periodic or
half-way bounce-back ends (mirror ghosts for rho and mu beyond a wall).

Coexistence follows from mu alone: the bulk phases of a planar equilibrium
have equal mu_b and equal p (Maxwell's construction).  Surface tension of a
planar interface: gamma = int k (d rho / dx)^2 dx = int sqrt(2 k omega(rho))
d rho over [rho_v, rho_l], omega(rho) = int_{rho_v}^{rho} (mu_b(s) - mu_0) ds
(the excess grand-potential density; k rho'^2 / 2 = omega is the first
integral of mu = mu_0), and the Laplace jump of a droplet is gamma / R in 2-D,
2 gamma / R in 3-D.
"""
from dataclasses import dataclass

import numpy as np
from scipy import integrate

from . import eos as eosmod
from . import step as S


# ---- bulk chemical potential of the equations of state ----

def mu_bulk(eos, rho):
    """mu_b(rho) with d mu_b / d rho = p'(rho) / rho, up to a constant: mu_b = phi/rho + p/rho, where
    phi / rho = int p / rho^2 d rho is the free energy per unit mass."""
    rho = np.asarray(rho, dtype=np.float64)
    if isinstance(eos, eosmod.PengRobinsonEOS):
        a, b, R, T, al = eos.a, eos.b, eos.R, eos.T, eos.alpha
        r2 = np.sqrt(2.0)
        # int p / rho^2: R T ln(rho / (1 - b rho)) - a alpha int d rho / (1 + 2 b rho - b^2 rho^2)
        f_per_mass = R * T * np.log(rho / (1.0 - b * rho)) - a * al / (2.0 * r2 * b) * np.log(
            (r2 - 1.0 + b * rho) / (r2 + 1.0 - b * rho))
    elif isinstance(eos, eosmod.PaperEOS):
        K, sv, rl = eos.K, np.sqrt(eos.rho_v), eos.rho_l
        f_per_mass = K * (rho ** 2 + (eos.rho_v - 2.0 * rl) * rho - 2.0 * sv * rho ** 1.5
                          + 4.0 * sv * rl * rho ** 0.5 - 2.0 * sv * rl ** 2 * rho ** -0.5)
    else:
        raise TypeError(type(eos))
    return f_per_mass + eos.p(rho) / rho


def omega_excess(eos, rho, rho_v, mu0):
    """omega(rho) = int_{rho_v}^{rho} (mu_b(s) - mu0) ds."""
    val, _ = integrate.quad(lambda s: mu_bulk(eos, s) - mu0, rho_v, rho, limit=400, epsabs=1e-15, epsrel=1e-12)
    return val


def gamma_planar(eos, k, rho_v, rho_l):
    """Surface tension of a planar interface between the coexisting densities rho_v, rho_l (Maxwell)."""
    mu0 = float(mu_bulk(eos, rho_v))
    val, _ = integrate.quad(lambda r: np.sqrt(max(2.0 * k * omega_excess(eos, r, rho_v, mu0), 0.0)), rho_v, rho_l,
                            limit=200, epsabs=1e-14, epsrel=1e-10)
    return val


# ---- the update ----

@dataclass
class WBParams:
    """A StepParams ``p`` (lattice, EOS, tau(rho), collision, walls, F_g) plus the gradient coefficient k and
    the reference density rho_0 of the well-balanced equilibrium."""
    p: object
    k: float
    rho0: float


def grad_d(lat, g, bcs):
    out = np.zeros((lat.d,) + g.shape)
    for i in range(lat.Q):
        gn = S.neighbour(lat, g, lat.c[i], bcs)
        for a in range(lat.d):
            if lat.c[i, a] != 0:
                out[a] += lat.w[i] * lat.c[i, a] * gn / lat.cs2
    return out


def lap_d(lat, g, bcs):
    out = np.zeros(g.shape)
    for i in range(lat.Q):
        gn = S.neighbour(lat, g, lat.c[i], bcs)
        out += lat.w[i] * (gn - g)
    return 2.0 * out / lat.cs2


def chemical_potential(wb, rho):
    p = wb.p
    return mu_bulk(p.eos, rho) - wb.k * lap_d(p.lat, rho, p.bcs())


def force(wb, rho):
    p = wb.p
    mu = chemical_potential(wb, rho)
    g = grad_d(p.lat, mu, p.bcs())
    return np.stack([-rho * g[a] + p.Fg[a] for a in range(p.lat.d)])


def equilibrium(lat, rho, u, rho0):
    """f_i^eq = w_i rho_0 + w_i rho s_i(u) (moving), f_0^eq = rho - (1 - w_0) rho_0 + w_0 rho s_0(u) (rest)."""
    cs2 = lat.cs2
    usq = sum(u[a] * u[a] for a in range(lat.d))
    feq = np.empty((lat.Q,) + rho.shape)
    for i in range(lat.Q):
        cu = sum(lat.c[i, a] * u[a] for a in range(lat.d))
        s_i = cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - usq / (2.0 * cs2)
        base = rho - (1.0 - lat.w[0]) * rho0 if i == 0 else lat.w[i] * rho0
        feq[i] = base + lat.w[i] * rho * s_i
    return feq


def macroscopic(wb, f):
    lat = wb.p.lat
    rho = S.density(f)
    F = force(wb, rho)
    u = (S.first_moment(lat, f) + 0.5 * F) / rho
    return rho, F, u


def step(wb, f):
    p = wb.p
    lat = p.lat
    rho, F, u = macroscopic(wb, f)
    tau = S.tau_of_rho(p, rho)
    feq = equilibrium(lat, rho, u, wb.rho0)
    Fhat = S.guo_source(lat, u, F)
    if p.collision == "bgk":
        fpost = S.collide_bgk(f, feq, Fhat, tau)
    else:
        fpost = S.collide_mrt(lat, f, feq, Fhat, tau, p.rates)
    return S.stream(lat, fpost, p.bcs())


def run(wb, f, n):
    for _ in range(n):
        f = step(wb, f)
    return f


def moments(wb, f):
    rho, _, u = macroscopic(wb, f)
    return rho, u


def init_equilibrium(wb, rho, u=None):
    lat = wb.p.lat
    rho = np.asarray(rho, dtype=np.float64)
    if u is None:
        u = np.zeros((lat.d,) + rho.shape)
    return equilibrium(lat, rho, np.asarray(u, dtype=np.float64), wb.rho0)
