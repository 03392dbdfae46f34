"""Shared set-up for the GPU parity tests: seeded inputs, oracle runs and the
library runs on the same inputs.  Each side derives its own lattice constants
from the same primary inputs (T/Tc, omega, eps, kappa, tau_v, tau_l, F_g).
"""
import functools
import sys

import numpy as np
import pytest

import plbm_synth as syn
from oracle import eos as E
from oracle import params as P
from oracle import step as S
from oracle.lattice import LATTICES


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    from paper_2504_15018_amd import native
    native.load()  # fails loudly when the HIP library is missing


@functools.lru_cache(maxsize=None)
def pr_coex(tr, omega=0.326, eps=2.0):
    return P.coexistence(E.PengRobinsonEOS(tr, omega), eps)


def oracle_params(lattice, tr=0.8, collision="bgk", walls=False, kappa=1.0, tau_v=1.0, tau_l=1.0,
                  Fg=(0.0, 0.0, 0.0), eps=2.0, rates=None):
    lat = LATTICES[lattice]
    rv, rl, _ = pr_coex(tr, 0.326, eps)
    bc = tuple("bb" if (walls and a == lat.d - 1) else "periodic" for a in range(lat.d))
    kw = {}
    if rates is not None:
        kw["rates"] = rates
    return S.StepParams(lat, E.PengRobinsonEOS(tr, 0.326), eps=eps, kappa=kappa, tau_v=tau_v, tau_l=tau_l,
                        rho_v=rv, rho_l=rl, Fg=tuple(Fg[: lat.d]) + (0.0,) * (3 - lat.d), collision=collision,
                        bc=bc, **kw)


def lib_params(tr=0.8, kappa=1.0, tau_v=1.0, tau_l=1.0, Fg=(0.0, 0.0, 0.0), eps=2.0):
    from paper_2504_15018_amd import native as N
    return N.plbm_params_pr_lattice(tr, 0.326, eps, kappa, tau_v, tau_l, list(Fg) + [0.0] * (3 - len(Fg)))


def random_state(lattice, dims, seed, tr=0.8, rel_amp=0.3):
    """Positive populations around a droplet density field (non-equilibrium)."""
    lat = LATTICES[lattice]
    rv, rl, _ = pr_coex(tr)
    co = syn.grid(dims)
    rho = syn.droplet(co, dims, rv, rl, R=min(dims) / 3.0, W=4.0, centre=[n / 2.0 - 0.3 for n in dims])
    return syn.random_populations(lat.Q, co, dims, seed, rho, rel_amp)


def fmt(name, **kw):
    s = name + " " + " ".join(f"{k}={v}" for k, v in kw.items())
    print(s, flush=True)
    sys.stdout.flush()
    return s


def tols(storage, steps):
    """Parity bars (relative on f and rho, absolute on u in lattice units) after `steps` steps.

    float64: 1e-12, 1e-12 (the oracle's own rounding is ~1e-16 per operation).
    float32: 1.5e-6 sqrt(steps) and 2e-7 sqrt(steps).  One update rounds each
    population through a chain of ~20 float32 operations (2^-24 each), and the
    roundings of successive steps are independent, so they add in quadrature;
    measured against the oracle: 1.1e-7 to 2.8e-7 relative on f and 8.8e-8 on
    u after 3-5 steps of random +-30 % states, 5.8e-6 and 6.0e-7 after 200
    steps of the 64^3 droplet (the bars leave 3-10x)."""
    if storage == "f64":
        return 1e-12, 1e-12
    r = max(steps, 1) ** 0.5
    return 1.5e-6 * r, 2e-7 * r


def rel_max(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def abs_max(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


# ---- 16-bit storage: the encoder's rounding reproduced on the host ----

ULP = {"f16s": 2.0**-11, "bf16s": 2.0**-8, "f16r": 2.0**-11, "bf16r": 2.0**-8}


def _bf16_round(x32):
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def _to16(x64, storage):
    x32 = x64.astype(np.float32)
    if storage.startswith("bf16"):
        return _bf16_round(x32).astype(np.float64)
    return x32.astype(np.float16).astype(np.float64)


def storage_round(lattice, f, storage, rho0):
    """The state f (Q, ...) as the encoder stores it, decoded back to float64."""
    w = LATTICES[lattice].w.reshape((-1,) + (1,) * (f.ndim - 1))
    if storage in ("f16s", "bf16s"):
        shift = w * rho0
    else:
        acc = f[0].copy()
        for q in range(1, f.shape[0]):
            acc = acc + f[q]
        ref = acc.astype(np.float32).astype(np.float16).astype(np.float64)
        shift = w * ref[None]
    return _to16(f - shift, storage) + shift
