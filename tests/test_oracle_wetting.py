"""Pins of the oracle's wetting walls (wall density rho_w sets the psi ghost
beyond a half-way bounce-back wall; an extension beyond the paper's solid walls).

Closed form, derived by hand for a uniform fluid (psi everywhere) next to a wall
whose ghost holds psi_w = psi + D: only the links that cross the wall see D.
Their weights sum to 1/6 on both D2Q9 and D3Q19, their c_a^2 (a lateral) to
1/18 and their c_a c_z to 0, so at the first fluid node
  M1 = -+ D/2 e_z,   M2 = diag(0, .., 0, D),   tr M2 = D,
the kappa terms cancel (M1.M2 = M1 tr M2) and
  F_z = +- (G psi D / 2 - G eps D^2 / 8)   (below: +, above: -),
with every other node and every lateral component force-free.
"""
import numpy as np
import pytest

from oracle import eos as E
from oracle import step as S
from oracle.lattice import LATTICES

from gpu_cases import oracle_params, random_state


def _uniform_force(lattice, dims, rho, rho_w, eps, kappa):
    op = oracle_params(lattice, walls=True, kappa=kappa)
    op.eps = eps
    op.rho_wall = rho_w
    shape = tuple(reversed(dims))
    psi = E.psi(op.eos, np.full(shape, rho))
    return op, psi, S.total_force(op, psi)


@pytest.mark.parametrize("lattice,dims", [("D2Q9", (6, 7)), ("D3Q19", (5, 4, 6))])
@pytest.mark.parametrize("eps,kappa", [(2.0, 1.0), (0.0, 1.7), (1.3, 0.6)])
def test_uniform_fluid_wall_force_closed_form(lattice, dims, eps, kappa):
    rho = 2.1
    op, psi, F = _uniform_force(lattice, dims, rho, (4.5, 0.9), eps, kappa)
    p = float(psi.flat[0])
    G = op.G
    d_lo = float(E.psi(op.eos, np.float64(4.5))) - p
    d_hi = float(E.psi(op.eos, np.float64(0.9))) - p
    zax = 0  # the wall axis is the slowest array axis in both layouts
    D = len(dims)
    Fz = np.moveaxis(F[D - 1], zax, 0)
    expect_lo = G * p * d_lo / 2.0 - G * eps * d_lo ** 2 / 8.0
    expect_hi = -(G * p * d_hi / 2.0 - G * eps * d_hi ** 2 / 8.0)
    scale = abs(p * d_lo)
    assert np.max(np.abs(Fz[0] - expect_lo)) <= 1e-14 * scale
    assert np.max(np.abs(Fz[-1] - expect_hi)) <= 1e-14 * scale
    assert np.max(np.abs(Fz[1:-1])) <= 1e-14 * scale
    for a in range(D - 1):
        assert np.max(np.abs(F[a])) <= 1e-14 * scale
    # a wall of the fluid's own density exerts no force
    _, _, F0 = _uniform_force(lattice, dims, rho, (rho, rho), eps, kappa)
    assert np.max(np.abs(F0)) <= 1e-14 * scale


def test_no_wall_density_is_the_mirror_ghost():
    """rho_w <= 0 keeps the neutral mirror ghost: identical to the default parameters."""
    lattice, dims = "D3Q19", (7, 5, 6)
    f0 = random_state(lattice, dims, 4)
    op = oracle_params(lattice, walls=True, collision="mrt")
    ref = S.run(op, f0, 3)
    op.rho_wall = (0.0, -1.0)
    assert np.array_equal(S.run(op, f0, 3), ref)
    op.rho_wall = (3.0, 0.0)  # a wetting wall below changes the result
    assert not np.array_equal(S.run(op, f0, 3), ref)


@pytest.mark.parametrize("lattice,dims", [("D2Q9", (9, 8)), ("D3Q19", (5, 6, 7))])
def test_wetting_walls_conserve_mass(lattice, dims):
    """The wall force is external (momentum changes) but bounce-back and the collision conserve mass."""
    f0 = random_state(lattice, dims, 6)
    op = oracle_params(lattice, walls=True, collision="mrt")
    op.rho_wall = (6.0, 0.4)
    f = S.run(op, f0, 10)
    assert abs(f.sum() - f0.sum()) <= 1e-13 * f0.sum()
    lat = LATTICES[lattice]
    j0 = S.first_moment(lat, f0).sum(axis=tuple(range(1, len(dims) + 1)))
    j1 = S.first_moment(lat, f).sum(axis=tuple(range(1, len(dims) + 1)))
    assert abs(j1[-1] - j0[-1]) > 1e-9  # the walls push along their normal
