"""Convenience wrapper around one libplbm lattice handle.

Owns a PyTorch uint8 device buffer as the lattice's memory and passes the
current HIP stream; everything else is argument marshalling to the C ABI.
Field arrays use the library's layout: (ny, nx) in 2-D, (nz, ny, nx) in 3-D.
"""
import numpy as np

from . import native as N

LATTICE = {"D2Q9": N.PLBM_D2Q9, "D3Q19": N.PLBM_D3Q19}
COLLISION = {"bgk": N.PLBM_BGK, "mrt": N.PLBM_MRT}
STORAGE = {"f64": N.PLBM_F64, "f32": N.PLBM_F32, "f16s": N.PLBM_F16S, "bf16s": N.PLBM_BF16S,
           "f16r": N.PLBM_F16R, "bf16r": N.PLBM_BF16R}
PATTERN = {"ab": N.PLBM_PATTERN_AB, "aa": N.PLBM_PATTERN_AA}
Q_OF = {"D2Q9": 9, "D3Q19": 19}


def make_desc(lattice, dims, collision="bgk", storage="f64", walls=False, rho0_shift=0.0, mrt_rates=None,
              pattern="ab", rho_wall=(0.0, 0.0), wb_k=0.0, wb_rho0=0.0):
    """dims = (nx, ny) for D2Q9 or (nx, ny, nz) for D3Q19; walls on the last axis;
    pattern "ab" (two population arrays) or "aa" (in place); rho_wall: wall
    densities below / above for wetting walls (0: neutral mirror); wb_k > 0
    selects the well-balanced scheme with that gradient coefficient (wb_rho0:
    its reference density, 0 = rho_v)."""
    d = N.plbm_lattice_desc()
    d.lattice = LATTICE[lattice]
    d.collision = COLLISION[collision]
    d.storage = STORAGE[storage]
    d.nx = dims[0]
    d.ny = dims[1]
    d.nz = dims[2] if len(dims) > 2 else 1
    last = len(dims) - 1
    for a in range(3):
        d.bc[a] = N.PLBM_HALFWAY_BB if (walls and a == last) else N.PLBM_PERIODIC
    d.pattern = PATTERN[pattern]
    d.rho_wall[0], d.rho_wall[1] = rho_wall
    d.rho0_shift = rho0_shift
    if wb_k > 0:
        d.scheme = N.PLBM_SCHEME_WELL_BALANCED
        d.wb_k = wb_k
        d.wb_rho0 = wb_rho0
    for k, v in enumerate(mrt_rates or (0.0, 0.0, 0.0, 0.0)):
        d.mrt_rates[k] = v
    return d


class Lattice:
    def __init__(self, lattice, dims, params, collision="bgk", storage="f64", walls=False, rho0_shift=0.0,
                 mrt_rates=None, stream=None, device="cuda", pattern="ab", rho_wall=(0.0, 0.0), wb_k=0.0,
                 wb_rho0=0.0):
        import torch

        self.name = lattice
        self.dims = tuple(int(v) for v in dims)
        self.D = len(self.dims)
        self.Q = Q_OF[lattice]
        self.N = int(np.prod(self.dims))
        self.shape = tuple(reversed(self.dims))
        self.desc = make_desc(lattice, dims, collision, storage, walls, rho0_shift, mrt_rates, pattern, rho_wall,
                              wb_k, wb_rho0)
        self.params = params
        self.nbytes = N.plbm_lattice_bytes(self.desc)
        self.mem = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        ptr = (self.mem.data_ptr() + 255) // 256 * 256
        # a dedicated stream (default priority) unless the caller passes one;
        # it can be captured into HIP graphs, unlike the legacy null stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.mem.device)
        self.h = N.plbm_create(self.desc, params, ptr, self.nbytes, self.stream.cuda_stream)

    def init_fields(self, rho, u=None):
        N.plbm_init_fields(self.h, np.asarray(rho).reshape(-1), None if u is None else np.asarray(u).reshape(-1))

    def init_shape(self, kind, rho_in, rho_out, W=5.0, R=0.0, centre=None, level=0.0, axis=0, u0=None):
        s = N.plbm_shape()
        s.kind, s.axis = kind, axis
        s.rho_in, s.rho_out, s.W, s.R, s.level = rho_in, rho_out, W, R, level
        for a, v in enumerate(centre or [n / 2.0 for n in self.dims]):
            s.centre[a] = v
        for a, v in enumerate(u0 or ()):
            s.u0[a] = v
        N.plbm_init_shape(self.h, s)

    def step(self, n=1):
        N.plbm_step(self.h, n)

    @property
    def time(self):
        return N.plbm_get_time(self.h)

    def moments(self):
        rho, u = N.plbm_read_moments(self.h, self.N, self.D)
        return rho.reshape(self.shape), u.reshape((self.D,) + self.shape)

    def populations(self):
        return N.plbm_read_populations(self.h, self.Q, self.N).reshape((self.Q,) + self.shape)

    def write_populations(self, f):
        N.plbm_write_populations(self.h, np.asarray(f).reshape(-1))

    def reduce(self, allow_unstable=False):
        return N.plbm_reduce(self.h, allow_unstable)

    def close(self):
        if getattr(self, "h", None):
            self.stream.synchronize()  # no kernel may still use the buffer when torch frees it
            N.plbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
