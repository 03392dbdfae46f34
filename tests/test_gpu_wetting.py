"""Wetting walls on the GPU (a wall density rho_w sets the psi ghost beyond a
half-way bounce-back wall; an extension beyond the paper's solid walls).

* Parity against the FP64 oracle with a different rho_w on each wall (same bars
  as the other parity tests), both storage patterns.
* Bitwise equality of the two storage patterns with wetting walls.
* Physics (checks that hold at any size): a 2-D droplet resting on the lower
  wall relaxes to a contact angle that decreases monotonically as rho_w rises
  from rho_v towards rho_l, and the neutral mirror ghost gives about 90 degrees.
  The angle comes from a least-squares circle through the mid-density contour
  away from the wall, intersected with the wall plane y = -1/2.

All cases run at T/Tc = 0.9 (density ratio 9.6).  A constant wall density is
stable over most of [rho_v, rho_l] there (angles 157 to 34 degrees for
rho_w = rho_v + 0.1 ... 0.7 (rho_l - rho_v), unstable at rho_l); at
T/Tc = 0.8 (ratio 31) only rho_w <= rho_v + 0.2 (rho_l - rho_v) is stable,
i.e. hydrophobic walls, and a wall density far above the adjacent vapour
drives |u| towards 1 within a few steps.
"""
import numpy as np
import pytest

from oracle import step as S

from gpu_cases import abs_max, fmt, lib_params, oracle_params, pr_coex, random_state, rel_max, require_gpu, tols

pytestmark = pytest.mark.gpu

TR = 0.9
CASES = [
    # lattice, dims, collision, storage, pattern, steps, rho_wall as fractions of (rho_v, rho_l)
    ("D2Q9", (40, 27), "mrt", "f64", "ab", 6, (0.4, 0.1)),
    ("D2Q9", (150, 21), "bgk", "f32", "aa", 5, (0.2, 0.3)),
    ("D3Q19", (37, 21, 13), "mrt", "f64", "aa", 5, (0.3, 0.0)),
    ("D3Q19", (70, 18, 11), "bgk", "f64", "ab", 4, (0.05, 0.35)),
    ("D3Q19", (35, 17, 10), "mrt", "f32", "ab", 3, (0.25, 0.15)),
]


def _rho_wall(frac, tr=TR):
    rv, rl, _ = pr_coex(tr)
    return tuple(0.0 if f == 0.0 else rv + f * (rl - rv) for f in frac)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[2]}-{c[3]}-{c[4]}-{c[6]}")
def test_wetting_walls_match_the_oracle(case):
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    lattice, dims, collision, storage, pattern, steps, frac = case
    fmt("wetting_oracle", case=case)
    rw = _rho_wall(frac)
    f0 = random_state(lattice, dims, 17, tr=TR)
    op = oracle_params(lattice, tr=TR, collision=collision, walls=True)
    op.rho_wall = rw
    lat = Lattice(lattice, dims, lib_params(tr=TR), collision=collision, storage=storage, walls=True,
                  pattern=pattern, rho_wall=rw)
    lat.write_populations(f0)
    if storage == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    lat.step(steps)
    f_ref = S.run(op, f0, steps)
    tf, tu = tols(storage, steps)
    assert rel_max(lat.populations(), f_ref) <= tf
    rho, u = lat.moments()
    rho_ref, u_ref = S.moments(op, f_ref)
    assert rel_max(rho, rho_ref) <= tf
    assert abs_max(u, u_ref) <= tu
    # the wall force acts: the same state with mirror walls differs
    op.rho_wall = (0.0, 0.0)
    assert rel_max(S.run(op, f0, steps), f_ref) > 1e-6
    lat.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16s"])
def test_wetting_walls_inplace_equals_ab_bitwise(storage):
    require_gpu()
    from paper_2504_15018_amd.lattice import Lattice
    fmt("wetting_inplace_vs_ab", storage=storage)
    dims = (70, 19, 13)
    rw = _rho_wall((0.3, 0.2))
    f0 = random_state("D3Q19", dims, 8, tr=TR)
    lats = [Lattice("D3Q19", dims, lib_params(tr=TR), collision="mrt", storage=storage, walls=True, pattern=p,
                    rho_wall=rw) for p in ("ab", "aa")]
    for lat in lats:
        lat.write_populations(f0)
        lat.step(11)
    fa, fb = lats[0].populations(), lats[1].populations()
    assert np.all(np.isfinite(fa)) and np.array_equal(fa, fb)
    for lat in lats:
        lat.close()


def _contact_angle(rho, rho_mid, y_min=6):
    """Circle through the mid-density contour (rows y >= y_min), intersected with the wall y = -1/2."""
    ny, nx = rho.shape
    pts = []
    for y in range(y_min, ny):
        row = rho[y] - rho_mid
        inside = np.nonzero(row > 0)[0]
        if inside.size == 0:
            break
        for x0, x1 in ((inside[0] - 1, inside[0]), (inside[-1], inside[-1] + 1)):
            a, b = row[x0 % nx], row[x1 % nx]
            pts.append((x0 + a / (a - b), float(y)))
    p = np.array(pts)
    # algebraic circle fit: x^2 + y^2 + D x + E y + F = 0
    A = np.column_stack([p[:, 0], p[:, 1], np.ones(len(p))])
    rhs = -(p[:, 0] ** 2 + p[:, 1] ** 2)
    D, E, F = np.linalg.lstsq(A, rhs, rcond=None)[0]
    xc, yc = -D / 2.0, -E / 2.0
    R = np.sqrt(xc * xc + yc * yc - F)
    return 90.0 + np.degrees(np.arcsin(np.clip((yc + 0.5) / R, -1.0, 1.0))), R


def test_contact_angle_follows_the_wall_density():
    require_gpu()
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    fmt("contact_angle")
    rv, rl, _ = pr_coex(TR)
    nx, ny = 240, 120
    prm = lib_params(tr=TR)
    angles = []
    for frac in (None, 0.1, 0.2, 0.3, 0.4, 0.5, 0.7):
        rw = 0.0 if frac is None else rv + frac * (rl - rv)
        lat = Lattice("D2Q9", (nx, ny), prm, collision="mrt", storage="f64", walls=True, rho_wall=(rw, 0.0))
        lat.init_shape(N.PLBM_SHAPE_DROPLET, rl, rv, W=5.0, R=36.0, centre=[nx / 2.0, 0.0])
        m0 = lat.reduce().mass
        lat.step(24000)
        d = lat.reduce()
        rho, _ = lat.moments()
        lat.close()
        assert d.flags == 0 and abs(d.mass - m0) <= 1e-10 * m0
        theta, R = _contact_angle(rho, 0.5 * (rv + rl), y_min=3)
        fmt("contact_angle_result", frac=frac, rho_w=f"{rw:.4f}", theta=f"{theta:.1f}", R=f"{R:.1f}",
            max_u=f"{d.max_u:.2e}")
        if frac is None:
            mirror = theta
        else:
            angles.append(theta)
    assert 85.0 <= mirror <= 95.0  # neutral wetting
    assert all(a > b + 8.0 for a, b in zip(angles, angles[1:])), angles  # monotone in rho_w
    assert angles[0] >= 140.0 and angles[-1] <= 50.0  # hydrophobic to hydrophilic


def test_contact_angle_3d_follows_the_wall_density():
    """D3Q19 sessile droplet (float64, MRT): the angle in the mid x-z plane orders like the 2-D one."""
    require_gpu()
    from paper_2504_15018_amd import native as N
    from paper_2504_15018_amd.lattice import Lattice
    fmt("contact_angle_3d")
    rv, rl, _ = pr_coex(TR)
    n, nz = 112, 56
    prm = lib_params(tr=TR)
    angles = {}
    for frac in (0.2, None, 0.5):
        rw = 0.0 if frac is None else rv + frac * (rl - rv)
        lat = Lattice("D3Q19", (n, n, nz), prm, collision="mrt", storage="f64", walls=True, rho_wall=(rw, 0.0))
        lat.init_shape(N.PLBM_SHAPE_DROPLET, rl, rv, W=5.0, R=24.0, centre=[n / 2.0, n / 2.0, 0.0])
        m0 = lat.reduce().mass
        lat.step(16000)
        d = lat.reduce()
        rho, _ = lat.moments()
        lat.close()
        assert d.flags == 0 and abs(d.mass - m0) <= 1e-10 * m0
        theta, R = _contact_angle(rho[:, n // 2, :], 0.5 * (rv + rl), y_min=3)  # (z, x) plane through the centre
        angles[frac] = theta
        fmt("contact_angle_3d_result", frac=frac, rho_w=f"{rw:.4f}", theta=f"{theta:.1f}", R=f"{R:.1f}",
            max_u=f"{d.max_u:.2e}")
    assert angles[0.2] > angles[None] + 8.0 > angles[0.5] + 16.0
    assert 80.0 <= angles[None] <= 100.0
