"""Grid convergence of the planar interface on the GPU (paper Sec. VI.A, Table II).

The paper's five grids: N_x = 100 ... 500 (N_y = N_x / 20, periodic), a
liquid slab in the central half, the paper EOS with rho_v = 0.0375,
rho_l = 1.187 in lattice units (R134a at 30 C with rho_l,lat = 1.187) and an
interface width of 150 nm, i.e. xi = 1.5 ... 7.5 lattice spacings.  Each grid
runs in float64 to equilibrium (max|u| below 1e-10); the whole density field
is compared with the Appendix A profile (interfaces placed at the simulated
mid-density crossings) through the relative L1, L2 and Linf norms of eq.
(relative_norms).  The paper reports second-order convergence of all three
norms in N_x; the fitted log-log slopes must be at least 1.8, and the vapour
and liquid bulk densities must approach rho_v and rho_l at second order too.
The equilibrium does not depend on tau (BGK, tau = 1 damps the slab's
acoustic modes fastest).
"""
import numpy as np
import pytest

from oracle import analytic as A
from oracle import norms as NO
from oracle import params as P

from gpu_cases import fmt, require_gpu

pytestmark = pytest.mark.gpu

RV, RL = 0.0375, 1.187
GRIDS = [(100, 5, 1.5), (200, 10, 3.0), (300, 15, 4.5), (400, 20, 6.0), (500, 25, 7.5)]


def _equilibrium(nx, ny, xi, max_steps=3_000_000, chunk=2000, tol=1e-10):
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    prm = N.plbm_params_paper_lattice(RV, RL, xi, 2.0, 1.0, 1.0, 1.0)
    lat = Lattice("D2Q9", (nx, ny), prm, collision="bgk", storage="f64")
    lat.init_shape(N.PLBM_SHAPE_SLAB, prm.rho_l, prm.rho_v, W=2.0 * xi, axis=0)
    steps = 0
    while steps < max_steps:
        lat.step(chunk)
        steps += chunk
        d = lat.reduce()
        if d.max_u < tol:
            break
    rho, _ = lat.moments()
    lat.close()
    return rho, steps, d.max_u


def test_planar_interface_second_order_on_the_paper_grids():
    require_gpu()
    L1, L2, Li, ev, el = [], [], [], [], []
    for nx, ny, xi in GRIDS:
        rho, steps, umax = _equilibrium(nx, ny, xi)
        assert np.all(rho == rho[:1, :])  # laterally uniform
        row = rho[0]
        K = P.K_from_width(xi, RV, RL)
        cr = A.mid_crossings(row, RV, RL)
        assert len(cr) == 2
        xl = [c for c, up in cr if up][0]
        xr = [c for c, up in cr if not up][0]
        x = np.arange(nx, dtype=np.float64)
        ana = np.where(np.abs(x - xl) < np.abs(x - xr), A.planar_profile(x, K, RV, RL, xl, rising=True),
                       A.planar_profile(x, K, RV, RL, xr, rising=False))
        n1, n2, ni = NO.relative_norms(np.broadcast_to(row, rho.shape), np.broadcast_to(ana, rho.shape))
        L1.append(n1)
        L2.append(n2)
        Li.append(ni)
        ev.append(abs(row.min() - RV) / RV)
        el.append(abs(row.max() - RL) / RL)
        fmt("planar_grid", nx=nx, xi=xi, steps=steps, max_u=f"{umax:.1e}", L1=f"{n1:.3e}", L2=f"{n2:.3e}",
            Linf=f"{ni:.3e}", rho_v_err=f"{ev[-1]:.3e}", rho_l_err=f"{el[-1]:.3e}")
    lx = np.log([g[0] for g in GRIDS])
    slopes = {name: -np.polyfit(lx, np.log(v), 1)[0] for name, v in
              (("L1", L1), ("L2", L2), ("Linf", Li), ("rho_v", ev), ("rho_l", el))}
    fmt("planar_orders", **{k: f"{v:.2f}" for k, v in slopes.items()})
    for k in ("L1", "L2", "Linf", "rho_v"):
        assert slopes[k] >= 1.8, (k, slopes[k])
