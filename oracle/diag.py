"""Global reductions of a lattice state (oracle, test infrastructure only).

Mass sum_x rho and momentum sum_x rho u (u including F/2, eq. Momentum) are
summed with math.fsum, i.e. correctly rounded, so they serve as the exact
reference for the library's compensated FP64 sums.  Health flags follow the
failure modes the paper names: a negative psi radicand (outside the
assumption p_EOS < rho c_s^2 of eq. Interaction_Potential), non-positive
density and non-finite values.
"""
import math

import numpy as np

from . import eos as eosmod
from .step import macroscopic

FLAG_NAN = 1
FLAG_RHO_NONPOS = 2
FLAG_PSI_NEG = 4


def exact_sum(a):
    return math.fsum(np.asarray(a, dtype=np.float64).ravel().tolist())


def reduce(p, f, u_prev=None, dt_prev=1):
    rho, psi, F, u = macroscopic(p, f)
    d = p.lat.d
    out = {
        "mass": exact_sum(rho),
        "momentum": [exact_sum(rho * u[a]) for a in range(d)],
        "max_u": float(np.max(np.sqrt(sum(u[a] * u[a] for a in range(d))))),
    }
    if u_prev is not None:
        du = np.sqrt(sum((u[a] - u_prev[a]) ** 2 for a in range(d)))
        out["max_du_per_step"] = float(np.max(du)) / dt_prev
    flags = 0
    if not (np.all(np.isfinite(f))):
        flags |= FLAG_NAN
    if np.any(rho <= 0):
        flags |= FLAG_RHO_NONPOS
    if np.any(eosmod.psi_radicand(p.eos, rho) < 0):
        flags |= FLAG_PSI_NEG
    out["flags"] = flags
    return out, u
