"""Equations of state and the pseudo-potential (oracle, test infrastructure only).

* Paper EOS, eq. (EOS) of Sec. IV:
      p = K [2 rho^3 + (rho_v - 2 rho_l) rho^2 - 3 sqrt(rho_v) rho^2.5
             + 2 sqrt(rho_v) rho_l rho^1.5 + sqrt(rho_v) rho_l^2 rho^0.5],
  with K = p_c / rho_c^3 and coexistence densities rho_v, rho_l by design.
* Peng-Robinson EOS (extension, not in the paper), in the lattice convention
  of Yuan and Schaefer (the paper's reference for eq. Interaction_Potential):
      p = rho R T / (1 - b rho) - a alpha(T) rho^2 / (1 + 2 b rho - b^2 rho^2),
  a = 2/49, b = 2/21, R = 1, alpha = [1 + m (1 - sqrt(T/Tc))]^2,
  m = 0.37464 + 1.54226 w - 0.26992 w^2 (w = acentric factor),
  Tc = 0.0778 a / (0.45724 b R).
* Pseudo-potential, eq. (Interaction_Potential) with G = -1 in lattice units:
      psi = sqrt(2 (rho/3 - p_EOS)).
  A negative radicand (outside the paper's assumption p_EOS < rho c_s^2) is
  clamped to zero and reported.
"""
from dataclasses import dataclass

import numpy as np

PR_A = 2.0 / 49.0
PR_B = 2.0 / 21.0
PR_R = 1.0
PR_OMEGA_COEF = (0.37464, 1.54226, -0.26992)


@dataclass
class PaperEOS:
    K: float
    rho_v: float
    rho_l: float

    def p(self, rho):
        rho = np.asarray(rho, dtype=np.float64)
        sv = np.sqrt(self.rho_v)
        rl = self.rho_l
        return self.K * (
            2.0 * rho ** 3
            + (self.rho_v - 2.0 * rl) * rho ** 2
            - 3.0 * sv * rho ** 2.5
            + 2.0 * sv * rl * rho ** 1.5
            + sv * rl ** 2 * rho ** 0.5
        )

    def p0(self):
        """Coexistence pressure p(rho_v) = p(rho_l) = K rho_l^2 rho_v."""
        return self.K * self.rho_l ** 2 * self.rho_v


@dataclass
class PengRobinsonEOS:
    T_over_Tc: float
    omega: float = 0.326
    a: float = PR_A
    b: float = PR_B
    R: float = PR_R

    @property
    def Tc(self):
        return 0.0778 * self.a / (0.45724 * self.b * self.R)

    @property
    def pc(self):
        return 0.0778 * self.R * self.Tc / self.b

    @property
    def T(self):
        return self.T_over_Tc * self.Tc

    @property
    def alpha(self):
        m = PR_OMEGA_COEF[0] + PR_OMEGA_COEF[1] * self.omega + PR_OMEGA_COEF[2] * self.omega ** 2
        return (1.0 + m * (1.0 - np.sqrt(self.T_over_Tc))) ** 2

    def p(self, rho):
        rho = np.asarray(rho, dtype=np.float64)
        a, b, R = self.a, self.b, self.R
        return rho * R * self.T / (1.0 - b * rho) - a * self.alpha * rho ** 2 / (
            1.0 + 2.0 * b * rho - b * b * rho ** 2
        )


def psi_radicand(eos, rho):
    """2 (rho/3 - p_EOS(rho)): the square of psi before clamping (G = -1)."""
    rho = np.asarray(rho, dtype=np.float64)
    return 2.0 * (rho / 3.0 - eos.p(rho))


def psi(eos, rho):
    """Pseudo-potential of eq. (Interaction_Potential), lattice units, G = -1."""
    return np.sqrt(np.maximum(psi_radicand(eos, rho), 0.0))
