"""Analytic references (oracle, test infrastructure only).

* Planar interface profile, Appendix A: sqrt(6 r K) x + C_0 = f_xi(rho).  The
  integration constant puts the mid density (rho_v + rho_l)/2 at a chosen
  position (one per interface).
* Surface tension of the paper EOS, Appendix B: gamma = sqrt(2K/(27 r)) kappa
  (f_gamma(rho_v) - f_gamma(rho_l)).
* Young-Laplace: Delta p = gamma / R in 2-D, 2 gamma / R in 3-D (Sec. VI.B).
* Two-phase channel (Sec. VI.D; the paper prints no formula): the steady 1-D
  momentum balance d/dy(mu du/dy) = -F_x with mu = rho nu(rho), nu linear in
  rho through tau(rho), no slip at the two walls; single-phase it is the
  Poiseuille parabola u = F y (H - y) / (2 mu).
"""
import numpy as np

from .params import f_xi, gamma_from_kappa  # noqa: F401  (re-exported)


def planar_profile(x, K, rho_v, rho_l, x_mid, r=1.0, rising=True):
    """rho(x) of Appendix A; ``rising`` = density increases with x."""
    x = np.asarray(x, dtype=np.float64)
    rho_m = 0.5 * (rho_v + rho_l)
    target = np.sqrt(6.0 * r * K) * ((x - x_mid) if rising else (x_mid - x)) + f_xi(rho_m, rho_v, rho_l)
    lo = np.full_like(x, rho_v)
    hi = np.full_like(x, rho_l)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        with np.errstate(invalid="ignore", divide="ignore"):
            val = f_xi(mid, rho_v, rho_l)
        go_up = val < target
        lo = np.where(go_up, mid, lo)
        hi = np.where(go_up, hi, mid)
    return 0.5 * (lo + hi)


def slab_profile(x, K, rho_v, rho_l, x_left, x_right, r=1.0):
    """Liquid slab between two interfaces centred at x_left < x_right."""
    x = np.asarray(x, dtype=np.float64)
    centre = 0.5 * (x_left + x_right)
    left = planar_profile(x, K, rho_v, rho_l, x_left, r, rising=True)
    right = planar_profile(x, K, rho_v, rho_l, x_right, r, rising=False)
    return np.where(x < centre, left, right)


def young_laplace(gamma, R, dim):
    return (dim - 1) * gamma / R


def mid_crossings(rho, rho_v, rho_l):
    """Positions (linear interpolation) where a periodic 1-D profile crosses the mid density."""
    rho = np.asarray(rho, dtype=np.float64)
    rho_m = 0.5 * (rho_v + rho_l)
    n = len(rho)
    out = []
    for i in range(n):
        a, b = rho[i] - rho_m, rho[(i + 1) % n] - rho_m
        if a == 0.0:
            out.append((float(i), b > 0 or rho[(i - 1) % n] < rho_m))
        elif a * b < 0:
            out.append((i + a / (a - b), b > 0))
    return out


def channel_velocity(y, rho_of_y, nu_of_rho, F, H, n_quad=20001):
    """u(y) solving d/dy(mu du/dy) = -F with u(0) = u(H) = 0, mu = rho nu(rho)."""
    s = np.linspace(0.0, H, n_quad)
    mu = rho_of_y(s) * nu_of_rho(rho_of_y(s))

    def cumtrapz(g):
        out = np.zeros_like(g)
        out[1:] = np.cumsum(0.5 * (g[1:] + g[:-1]) * np.diff(s))
        return out

    I1 = cumtrapz(1.0 / mu)
    I2 = cumtrapz(s / mu)
    C = F * I2[-1] / I1[-1]
    u_s = C * I1 - F * I2
    return np.interp(y, s, u_s)


def poiseuille(y, F, mu, H):
    y = np.asarray(y, dtype=np.float64)
    return F * y * (H - y) / (2.0 * mu)
