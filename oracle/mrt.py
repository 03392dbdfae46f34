"""Moment bases for the multiple-relaxation-time collision (extension, not in
the paper; oracle, test infrastructure only).

The paper uses BGK only (Sec. II, eq. LBE).  The MRT variant keeps every other
part of the update and relaxes moments m = M f instead of populations:

    m* = m - S (m - m_eq) + (I - S/2) M Fhat,      f* = M^-1 m*,

with m_eq = M f_eq (projection of the same second-order equilibrium) and
Fhat_i = w_i [c.F / cs^2 + (c.u)(c.F)/cs^4 - (u.F)/cs^2] (Guo's source without
its (1 - 1/(2 tau)) prefactor).  With every rate equal to 1/tau this is BGK.

Bases (rows are orthogonal, so M^-1 = M^T diag(1/|row|^2)):
  D2Q9  (Lallemand-Luo): 1, 3|c|^2-4, (9|c|^4-21|c|^2+8)/2, cx, (3|c|^2-5)cx,
                          cy, (3|c|^2-5)cy, cx^2-cy^2, cx cy
  D3Q19 (d'Humieres):    1, 19|c|^2-30, (21|c|^4-53|c|^2+24)/2,
                          cx, (5|c|^2-9)cx, cy, (5|c|^2-9)cy, cz, (5|c|^2-9)cz,
                          3cx^2-|c|^2, (3|c|^2-5)(3cx^2-|c|^2),
                          cy^2-cz^2, (3|c|^2-5)(cy^2-cz^2),
                          cx cy, cy cz, cx cz,
                          (cy^2-cz^2)cx, (cz^2-cx^2)cy, (cx^2-cy^2)cz
Rate classes per row (the names select entries of a rates dict):
  'rho' (conserved), 'e', 'eps', 'j', 'q', 'nu' (stress; = 1/tau(rho)),
  'pi' (D3Q19 only; defaults to the stress rate), 'm' (D3Q19 only).
"""
import numpy as np

from .lattice import D2Q9, D3Q19


def _rows_d2q9(c):
    cx, cy = c[:, 0].astype(np.float64), c[:, 1].astype(np.float64)
    c2 = cx * cx + cy * cy
    rows = [
        np.ones_like(cx),
        3 * c2 - 4,
        (9 * c2 * c2 - 21 * c2 + 8) / 2,
        cx,
        (3 * c2 - 5) * cx,
        cy,
        (3 * c2 - 5) * cy,
        cx * cx - cy * cy,
        cx * cy,
    ]
    classes = ["rho", "e", "eps", "j", "q", "j", "q", "nu", "nu"]
    return np.array(rows), classes


def _rows_d3q19(c):
    cx, cy, cz = (c[:, k].astype(np.float64) for k in range(3))
    c2 = cx * cx + cy * cy + cz * cz
    rows = [
        np.ones_like(cx),
        19 * c2 - 30,
        (21 * c2 * c2 - 53 * c2 + 24) / 2,
        cx,
        (5 * c2 - 9) * cx,
        cy,
        (5 * c2 - 9) * cy,
        cz,
        (5 * c2 - 9) * cz,
        3 * cx * cx - c2,
        (3 * c2 - 5) * (3 * cx * cx - c2),
        cy * cy - cz * cz,
        (3 * c2 - 5) * (cy * cy - cz * cz),
        cx * cy,
        cy * cz,
        cx * cz,
        (cy * cy - cz * cz) * cx,
        (cz * cz - cx * cx) * cy,
        (cx * cx - cy * cy) * cz,
    ]
    classes = ["rho", "e", "eps", "j", "q", "j", "q", "j", "q",
               "nu", "pi", "nu", "pi", "nu", "nu", "nu", "m", "m", "m"]
    return np.array(rows), classes


def basis(lat):
    """Return (M, M_inv, classes) for the lattice."""
    if lat is D2Q9:
        M, classes = _rows_d2q9(lat.c)
    elif lat is D3Q19:
        M, classes = _rows_d3q19(lat.c)
    else:
        raise ValueError(lat)
    norms = np.sum(M * M, axis=1)
    M_inv = M.T / norms[None, :]
    return M, M_inv, classes


DEFAULT_RATES = {"e": 0.8, "eps": 0.8, "q": 1.1, "m": 1.1, "j": 1.0, "rho": 1.0}
