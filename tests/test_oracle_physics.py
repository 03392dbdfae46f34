"""Physics pins of the oracle on small lattices (Sec. VI benchmarks, scaled down).

* Planar interface (Sec. VI.A): the equilibrium densities approach the
  mechanical-stability prediction of Sec. IV at second order in the interface
  width, and the profile approaches Appendix A.
* With the eps coefficient as printed in eq. (interactionForce) the planar
  interface does not reach that prediction (documents the reading of the eps
  term, see ``oracle.step``).
* Young-Laplace (Sec. VI.B): Delta p R of a 2-D droplet is close to the
  predicted surface tension and scales with kappa.
"""
import numpy as np
import pytest

import plbm_synth as syn
from oracle import analytic as A
from oracle import eos as E
from oracle import params as P
from oracle import step as S
from oracle.lattice import D2Q9

RV, RL = 0.0375, 1.187


def _planar(xi, nx, force_form="consistent", max_steps=30000, tol=1e-9, tau=1.5):
    K = P.K_from_width(xi, RV, RL)
    e = E.PaperEOS(K, RV, RL)
    cv, cl, p0 = P.coexistence(e, 2.0, rho_hi=3.0)
    x = np.arange(nx, dtype=np.float64)
    rho0 = A.slab_profile(x, K, cv, cl, nx / 4, 3 * nx / 4)[None, :]
    # the equilibrium does not depend on tau; tau = 1.5 damps the slab's acoustic modes faster
    p = S.StepParams(D2Q9, e, eps=2.0, kappa=1.0, tau_v=tau, tau_l=tau, rho_v=cv, rho_l=cl,
                     force_form=force_form)
    f = S.init_equilibrium(D2Q9, rho0)
    steps = 0
    while steps < max_steps:
        f = S.run(p, f, 1000)
        steps += 1000
        rho, u = S.moments(p, f)
        if not np.all(np.isfinite(rho)):
            return None, (cv, cl), K
        if np.max(np.abs(u)) < tol:
            break
    return rho[0], (cv, cl), K


@pytest.mark.slow
def test_planar_interface_second_order():
    errs_v, errs_l, prof = [], [], []
    # the vapour gap must hold many tail lengths 1/(sqrt(6K)(rho_l - rho_v)) ~ 1.1 xi
    for xi, nx in ((1.5, 64), (3.0, 128)):
        rho, (cv, cl), K = _planar(xi, nx)
        assert rho is not None
        errs_v.append(abs(rho.min() - cv) / cv)
        errs_l.append(abs(rho.max() - cl) / cl)
        # whole-profile error against Appendix A (interfaces placed at the simulated crossings)
        cr = A.mid_crossings(rho, RV, RL)
        assert len(cr) == 2
        xl = [c for c, up in cr if up][0]
        xr = [c for c, up in cr if not up][0]
        x = np.arange(nx, dtype=np.float64)
        ana = np.where(np.abs(x - xl) < np.abs(x - xr),
                       A.planar_profile(x, K, RV, RL, xl, rising=True),
                       A.planar_profile(x, K, RV, RL, xr, rising=False))
        prof.append(np.sqrt(np.sum((rho - ana) ** 2) / np.sum(ana ** 2)))
    # vapour density within a few percent of the prediction, error shrinking ~ xi^-2
    assert errs_v[0] < 0.05 and errs_v[1] < 0.015
    assert 3.0 < errs_v[0] / errs_v[1] < 5.0
    assert errs_l[1] < errs_l[0] < 2e-3
    assert prof[1] < prof[0] / 2.5


@pytest.mark.slow
def test_printed_eps_coefficient_misses_the_prediction():
    rho, (cv, cl), _ = _planar(1.5, 64, force_form="printed", max_steps=6000, tol=0.0)
    ok, _, _ = _planar(1.5, 64, max_steps=6000, tol=0.0)
    if rho is not None:
        # far further from the mechanical-stability prediction than the consistent form
        assert abs(rho.min() - cv) / cv > 5 * abs(ok.min() - cv) / cv


@pytest.mark.slow
def test_young_laplace_and_kappa_scaling():
    xi = 1.5
    K = P.K_from_width(xi, RV, RL)
    e = E.PaperEOS(K, RV, RL)
    cv, cl, p0 = P.coexistence(e, 2.0, rho_hi=3.0)
    gk = P.gamma_over_kappa_general(e, cv, cl, p0)
    n = 40
    dims = (n, n)
    co = syn.grid(dims)
    out = {}
    for kappa in (1.0, 2.0):
        p = S.StepParams(D2Q9, e, eps=2.0, kappa=kappa, tau_v=1.0, tau_l=1.0, rho_v=cv, rho_l=cl)
        rho0 = syn.droplet(co, dims, cv, cl, R=10.0, W=3.0)
        f = S.run(p, S.init_equilibrium(D2Q9, rho0), 6000)
        rho, u = S.moments(p, f)
        r_in, r_out = rho[n // 2, n // 2], rho[0, 0]
        dp = e.p(r_in) - e.p(r_out)
        area = np.sum((rho - r_out) / (r_in - r_out))
        R = np.sqrt(area / np.pi)
        out[kappa] = (dp * R, np.max(np.sqrt(u[0] ** 2 + u[1] ** 2)))
    assert out[1.0][0] == pytest.approx(gk * 1.0, rel=0.15)
    assert out[2.0][0] / out[1.0][0] == pytest.approx(2.0, rel=0.1)
    # spurious currents: small but non-zero, as in Sec. VI.B
    assert 0 < out[1.0][1] < 1e-2
