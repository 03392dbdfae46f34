"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module generates INPUTS only: initial density fields shaped like the
paper's benchmark problems (planar slab, static droplet, layered channel),
small seeded perturbations, uniform or random velocity fields, positive random
population sets, and the request stream of the serving workload.  It holds
none of the lattice Boltzmann arithmetic: no weights, no equilibria, no EOS.

Every generator is a function of integer lattice coordinates, so a window of
a large lattice (with periodic wrap) yields exactly the values of the full
array at those coordinates.  Random values come from a counter-based hash
(SplitMix64 finaliser applied to seed, stream and site index), not from a
stateful generator.

Field arrays use the library's layout: (ny, nx) in 2-D, (nz, ny, nx) in 3-D,
x fastest.  ``dims`` is always given as (nx, ny[, nz]).
"""
import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(z):
    z = z.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed, stream, index):
    """Counter-based uniform numbers in [0, 1) for integer site indices."""
    index = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = _splitmix64(np.uint64(seed) * np.uint64(0x100000001B3) + np.uint64(stream))
        z = _splitmix64(index ^ key)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def grid(dims):
    """Coordinate arrays (x, y[, z]) in field layout for a lattice of size dims."""
    axes = [np.arange(n) for n in reversed(dims)]
    mesh = np.meshgrid(*axes, indexing="ij")  # (z, y, x) or (y, x)
    return tuple(reversed(mesh))


def linear_index(coords, dims):
    """x + nx (y + ny z) of (possibly wrapped) coordinates."""
    idx = np.zeros(np.shape(coords[0]), dtype=np.int64)
    stride = 1
    for c, n in zip(coords, dims):
        idx = idx + (np.asarray(c) % n) * stride
        stride *= n
    return idx


# ----------------------------------------------------------------------------
# density shapes (tanh interfaces of width W)

def slab(coords, dims, rho_v, rho_l, W=5.0, axis=0):
    """Liquid slab in the central half along ``axis`` (interfaces at n/4, 3n/4)."""
    n = dims[axis]
    x = np.asarray(coords[axis], dtype=np.float64)
    return rho_v + 0.5 * (rho_l - rho_v) * (np.tanh(2.0 * (x - n / 4.0) / W) - np.tanh(2.0 * (x - 3.0 * n / 4.0) / W))


def droplet(coords, dims, rho_v, rho_l, R, W=5.0, centre=None):
    """Liquid droplet of radius R, centred at dims/2 unless given."""
    if centre is None:
        centre = [n / 2.0 for n in dims]
    r2 = 0.0
    for c, c0 in zip(coords, centre):
        r2 = r2 + (np.asarray(c, dtype=np.float64) - c0) ** 2
    d = np.sqrt(r2)
    return 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (d - R) / W)


def layers(coords, dims, rho_v, rho_l, W=5.0, axis=None, level=None):
    """Liquid below ``level`` along ``axis`` (default: last axis, half height)."""
    if axis is None:
        axis = len(dims) - 1
    if level is None:
        level = dims[axis] / 2.0
    z = np.asarray(coords[axis], dtype=np.float64)
    return 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (z - level) / W)


def perturb(rho, coords, dims, seed, rel_amp):
    """rho (1 + rel_amp (2U - 1)) with counter-based U per site."""
    u = uniform01(seed, 7, linear_index(coords, dims))
    return rho * (1.0 + rel_amp * (2.0 * u - 1.0))


def random_velocity(coords, dims, seed, amp):
    """Components in [-amp, amp], shape (d,) + field shape."""
    idx = linear_index(coords, dims)
    return np.stack([amp * (2.0 * uniform01(seed, 100 + a, idx) - 1.0) for a in range(len(dims))])


def uniform_velocity(coords, u0):
    shape = np.shape(coords[0])
    return np.stack([np.full(shape, float(v)) for v in u0])


def random_populations(Q, coords, dims, seed, rho, rel_amp=0.3):
    """Q positive values per site, each rho/Q (1 + rel_amp (2U - 1)).

    These are arbitrary non-equilibrium states for parity tests; they carry no
    lattice weights.
    """
    idx = linear_index(coords, dims)
    return np.stack([rho / Q * (1.0 + rel_amp * (2.0 * uniform01(seed, 1000 + i, idx) - 1.0)) for i in range(Q)])


def window(dims, lo, size):
    """Wrapped coordinates of a box [lo, lo + size) on a periodic lattice."""
    axes = [(np.arange(s) + l) % n for l, s, n in zip(lo, size, dims)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")
    return tuple(reversed(mesh))


# ----------------------------------------------------------------------------
# serving workload: a Poisson stream of uneven requests

def request_stream(n, rate, seed=0, side2d=(64, 1024), side3d=(64, 192), t_range=(0.6, 0.9), r_frac=(0.15, 0.35),
                   channel_frac=0.0, width2d=(64, 512), width3d=(64, 192), channel_len=8, body_force=1e-6):
    """List of dicts: arrival time, lattice type, sides, T/Tc, and the problem: a static droplet (radius), or,
    with probability channel_frac, a two-phase channel between walls on the last axis (width = that axis,
    channel_len nodes along the others, body force along x).  The droplet draws do not depend on
    channel_frac."""
    k = np.arange(n, dtype=np.uint64)
    gaps = -np.log(1.0 - uniform01(seed, 1, k)) / rate
    arrivals = np.cumsum(gaps)
    kind = uniform01(seed, 2, k) < 0.5
    u_side = uniform01(seed, 3, k)
    u_t = uniform01(seed, 4, k)
    u_r = uniform01(seed, 5, k)
    chan = uniform01(seed, 6, k) < channel_frac
    out = []
    for i in range(n):
        lo, hi = (width2d if kind[i] else width3d) if chan[i] else (side2d if kind[i] else side3d)
        side = int(lo + np.floor(u_side[i] * (hi - lo + 1)))
        if chan[i]:
            dims = (channel_len, side) if kind[i] else (channel_len, channel_len, side)
        else:
            dims = (side, side) if kind[i] else (side, side, side)
        out.append({
            "id": i,
            "arrival": float(arrivals[i]),
            "lattice": "D2Q9" if kind[i] else "D3Q19",
            "dims": dims,
            "T_over_Tc": float(t_range[0] + u_t[i] * (t_range[1] - t_range[0])),
            "radius": 0.0 if chan[i] else float((r_frac[0] + u_r[i] * (r_frac[1] - r_frac[0])) * side),
            "problem": "channel" if chan[i] else "droplet",
            "body_force": float(body_force) if chan[i] else 0.0,
        })
    return out
