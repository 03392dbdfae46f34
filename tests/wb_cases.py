"""Test helper: the discrete equilibrium of the well-balanced scheme's lattice
equations (uniform lattice chemical potential at fixed mass), by Newton's
method on the oracle's bulk chemical potential and the isotropic D2Q9
Laplacian.  Independent of the update itself; used to pin the oracle and to
give the GPU a state that must stay fixed."""
import numpy as np
from scipy import sparse
from scipy.sparse.linalg import spsolve

from oracle import wellbalanced as W
from oracle.lattice import D2Q9


def lap_matrix(dims):
    """lap_d on a periodic 2-D lattice as a sparse matrix (field index y * nx + x)."""
    nx, ny = dims
    n = nx * ny
    idx = np.arange(n)
    x, y = idx % nx, idx // nx
    rows, cols, vals = [], [], []
    for i in range(1, 9):
        cx, cy = D2Q9.c[i]
        j = ((y + cy) % ny) * nx + (x + cx) % nx
        rows += [idx, idx]
        cols += [j, idx]
        vals += [np.full(n, 2.0 * D2Q9.w[i] / D2Q9.cs2), np.full(n, -2.0 * D2Q9.w[i] / D2Q9.cs2)]
    return sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def discrete_equilibrium(eos, k, rho_init, iters=40):
    """Newton's method on mu_b(rho) - k lap_d rho = mu0 at every node with the total mass fixed (unknowns:
    rho and mu0).  Returns the density field."""
    ny, nx = rho_init.shape
    n = nx * ny
    Lm = lap_matrix((nx, ny))
    rho = rho_init.ravel().copy()
    mass = rho.sum()
    mu0 = float(np.mean(W.mu_bulk(eos, rho)))
    for _ in range(iters):
        mu = W.mu_bulk(eos, rho) - k * (Lm @ rho)
        res = np.concatenate([mu - mu0, [rho.sum() - mass]])
        if np.max(np.abs(res)) < 1e-15:
            break
        h = 1e-7 * rho
        dmu = (W.mu_bulk(eos, rho + h) - W.mu_bulk(eos, rho - h)) / (2 * h)
        J = sparse.bmat([[sparse.diags(dmu) - k * Lm, -np.ones((n, 1))], [np.ones((1, n)), None]], format="csc")
        d = spsolve(J, -res)
        rho = rho + d[:n]
        mu0 = mu0 + d[n]
    return rho.reshape(ny, nx)
