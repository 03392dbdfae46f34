"""ctypes binding of libplbm (include/plbm.h): argument marshalling only.

Every step of the lattice update runs in the library's HIP kernels.  PyTorch
supplies device memory (uint8 tensors) and the current HIP stream.  Loading
fails loudly when the library has not been built; there is no fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libplbm.so")

# ---- constants (plbm.h) ----
PLBM_ABI_VERSION = 4
PLBM_OK = 0
PLBM_E_INVALID = -1
PLBM_E_UNSUPPORTED = -2
PLBM_E_NOMEM = -3
PLBM_E_DEVICE = -4
PLBM_E_UNSTABLE = -5
PLBM_E_NOCONVERGE = -6
PLBM_D2Q9, PLBM_D3Q19 = 0, 1
PLBM_BGK, PLBM_MRT = 0, 1
PLBM_F64, PLBM_F32, PLBM_F16S, PLBM_BF16S, PLBM_F16R, PLBM_BF16R = 0, 1, 2, 3, 4, 5
PLBM_PERIODIC, PLBM_HALFWAY_BB = 0, 1
PLBM_PATTERN_AB, PLBM_PATTERN_AA = 0, 1
PLBM_SCHEME_PSEUDOPOTENTIAL, PLBM_SCHEME_WELL_BALANCED = 0, 1
PLBM_EOS_PAPER, PLBM_EOS_PENG_ROBINSON = 0, 1
PLBM_FLAG_NAN, PLBM_FLAG_RHO_NONPOS, PLBM_FLAG_PSI_NEG = 1, 2, 4
PLBM_SHAPE_SLAB, PLBM_SHAPE_DROPLET, PLBM_SHAPE_LAYERS = 0, 1, 2

_D = ctypes.c_double
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)


class plbm_phys_params(ctypes.Structure):
    _fields_ = [("eos", _I32), ("pad0", _I32), ("rho_v", _D), ("rho_l", _D), ("nu_v", _D), ("nu_l", _D),
                ("gamma", _D), ("xi", _D), ("L", _D), ("body_force", _D * 3), ("T_over_Tc", _D), ("omega", _D),
                ("epsilon", _D), ("U_phys", _D)]


class plbm_lattice_map(ctypes.Structure):
    _fields_ = [("L_lat", _D), ("tau_l", _D), ("rho_l_lat", _D)]


class plbm_lattice_params(ctypes.Structure):
    _fields_ = [("eos", _I32), ("pad0", _I32), ("K", _D), ("eos_rho_v", _D), ("eos_rho_l", _D), ("pr_a", _D),
                ("pr_b", _D), ("pr_R", _D), ("pr_T", _D), ("pr_alpha", _D), ("rho_v", _D), ("rho_l", _D),
                ("epsilon", _D), ("kappa", _D), ("G", _D), ("tau_v", _D), ("tau_l", _D), ("body_force", _D * 3),
                ("C_L", _D), ("C_T", _D), ("C_M", _D), ("C_U", _D), ("C_VF", _D), ("C_gamma", _D), ("C_p", _D),
                ("Re", _D), ("gamma_lat", _D)]


class plbm_lattice_desc(ctypes.Structure):
    _fields_ = [("lattice", _I32), ("collision", _I32), ("storage", _I32), ("nx", _I32), ("ny", _I32),
                ("nz", _I32), ("bc", _I32 * 3), ("pattern", _I32), ("rho0_shift", _D), ("mrt_rates", _D * 4),
                ("rho_wall", _D * 2), ("scheme", _I32), ("pad1", _I32), ("wb_k", _D), ("wb_rho0", _D)]


class plbm_shape(ctypes.Structure):
    _fields_ = [("kind", _I32), ("axis", _I32), ("rho_in", _D), ("rho_out", _D), ("W", _D), ("R", _D),
                ("centre", _D * 3), ("level", _D), ("u0", _D * 3)]


class plbm_diag(ctypes.Structure):
    _fields_ = [("mass", _D), ("mass_comp_err", _D), ("momentum", _D * 3), ("max_u", _D),
                ("max_du_per_step", _D), ("time", _I64), ("flags", _I32), ("pad0", _I32)]


_SIGS = {
    "plbm_abi_version": (ctypes.c_int, []),
    "plbm_last_error": (ctypes.c_char_p, []),
    "plbm_resolve_params": (ctypes.c_int, [ctypes.POINTER(plbm_phys_params), ctypes.POINTER(plbm_lattice_map),
                                           ctypes.POINTER(plbm_lattice_params)]),
    "plbm_params_pr_lattice": (ctypes.c_int, [_D, _D, _D, _D, _D, _D, _DP, ctypes.POINTER(plbm_lattice_params)]),
    "plbm_params_paper_lattice": (ctypes.c_int, [_D, _D, _D, _D, _D, _D, _D, _DP,
                                                 ctypes.POINTER(plbm_lattice_params)]),
    "plbm_lattice_bytes": (ctypes.c_int, [ctypes.POINTER(plbm_lattice_desc), ctypes.POINTER(_U64)]),
    "plbm_create": (ctypes.c_int, [ctypes.POINTER(plbm_lattice_desc), ctypes.POINTER(plbm_lattice_params), _VP,
                                   _U64, _VP, ctypes.POINTER(_VP)]),
    "plbm_init_fields": (ctypes.c_int, [_VP, _DP, _DP]),
    "plbm_init_shape": (ctypes.c_int, [_VP, ctypes.POINTER(plbm_shape)]),
    "plbm_step": (ctypes.c_int, [_VP, _I64]),
    "plbm_read_moments": (ctypes.c_int, [_VP, _DP, _DP]),
    "plbm_moments_device": (ctypes.c_int, [_VP, _VP, _VP]),
    "plbm_read_populations": (ctypes.c_int, [_VP, _DP]),
    "plbm_write_populations": (ctypes.c_int, [_VP, _DP]),
    "plbm_get_time": (ctypes.c_int, [_VP, ctypes.POINTER(_I64)]),
    "plbm_reduce": (ctypes.c_int, [_VP, ctypes.POINTER(plbm_diag)]),
    "plbm_reduce_static": (ctypes.c_int, [_VP, ctypes.POINTER(plbm_diag)]),
    "plbm_destroy": (None, [_VP]),
    "plbm_batch_bytes": (ctypes.c_int, [_I32, _I64, ctypes.POINTER(_U64)]),
    "plbm_batch_create": (ctypes.c_int, [_I32, _I64, _VP, _U64, _VP, ctypes.POINTER(_VP)]),
    "plbm_batch_attach": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(_I32)]),
    "plbm_batch_detach": (ctypes.c_int, [_VP, _I32]),
    "plbm_batch_step": (ctypes.c_int, [_VP, _I64]),
    "plbm_batch_diag": (ctypes.c_int, [_VP, ctypes.POINTER(plbm_diag)]),
    "plbm_batch_destroy": (None, [_VP]),
}

EXPORTED = tuple(_SIGS)

_lib = None


class PlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libplbm error {code}: {msg}")
        self.code = code


def load(path=None):
    """Load libplbm (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  (loads the HIP runtime the library links against)
    except ImportError:
        pass
    p = path or os.environ.get("PLBM_LIB") or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built: run `python -m paper_2504_15018_amd.build` (the HIP library is "
                           "required; there is no CPU fallback)")
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.plbm_abi_version() != PLBM_ABI_VERSION:
        raise RuntimeError("libplbm ABI version mismatch")
    _lib = lib
    return lib


def check(code):
    if code != PLBM_OK:
        raise PlbmError(code, load().plbm_last_error().decode())
    return code


def _dptr(a):
    return a.ctypes.data_as(_DP) if a is not None else None


# ---- one Python function per C entry point (same names) ----

def plbm_abi_version():
    return load().plbm_abi_version()


def plbm_last_error():
    return load().plbm_last_error().decode()


def plbm_resolve_params(phys, lmap):
    out = plbm_lattice_params()
    check(load().plbm_resolve_params(ctypes.byref(phys), ctypes.byref(lmap), ctypes.byref(out)))
    return out


def plbm_params_pr_lattice(T_over_Tc, omega=0.326, epsilon=2.0, kappa=1.0, tau_v=1.0, tau_l=1.0, body_force=None):
    out = plbm_lattice_params()
    bf = (_D * 3)(*body_force) if body_force is not None else None
    check(load().plbm_params_pr_lattice(T_over_Tc, omega, epsilon, kappa, tau_v, tau_l, bf, ctypes.byref(out)))
    return out


def plbm_params_paper_lattice(rho_v, rho_l, xi, epsilon=2.0, kappa=1.0, tau_v=1.0, tau_l=1.0, body_force=None):
    out = plbm_lattice_params()
    bf = (_D * 3)(*body_force) if body_force is not None else None
    check(load().plbm_params_paper_lattice(rho_v, rho_l, xi, epsilon, kappa, tau_v, tau_l, bf, ctypes.byref(out)))
    return out


def plbm_lattice_bytes(desc):
    n = _U64()
    check(load().plbm_lattice_bytes(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def plbm_create(desc, params, dev_ptr, dev_bytes, stream_ptr):
    h = _VP()
    check(load().plbm_create(ctypes.byref(desc), ctypes.byref(params), dev_ptr, dev_bytes, stream_ptr,
                             ctypes.byref(h)))
    return h.value


def plbm_init_fields(h, rho, u=None):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    check(load().plbm_init_fields(h, _dptr(rho), _dptr(u)))


def plbm_init_shape(h, shape):
    check(load().plbm_init_shape(h, ctypes.byref(shape)))


def plbm_step(h, n):
    check(load().plbm_step(h, int(n)))


def plbm_read_moments(h, N, D):
    rho = np.empty(N, dtype=np.float64)
    u = np.empty(D * N, dtype=np.float64)
    check(load().plbm_read_moments(h, _dptr(rho), _dptr(u)))
    return rho, u


def plbm_moments_device(h, rho_dev_ptr, u_dev_ptr):
    check(load().plbm_moments_device(h, rho_dev_ptr, u_dev_ptr))


def plbm_read_populations(h, Q, N):
    f = np.empty(Q * N, dtype=np.float64)
    check(load().plbm_read_populations(h, _dptr(f)))
    return f


def plbm_write_populations(h, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    check(load().plbm_write_populations(h, _dptr(f)))


def plbm_get_time(h):
    t = _I64()
    check(load().plbm_get_time(h, ctypes.byref(t)))
    return t.value


def plbm_reduce(h, allow_unstable=False):
    d = plbm_diag()
    code = load().plbm_reduce(h, ctypes.byref(d))
    if code != PLBM_OK and not (allow_unstable and code == PLBM_E_UNSTABLE):
        check(code)
    return d


def plbm_reduce_static(h, allow_unstable=False):
    d = plbm_diag()
    code = load().plbm_reduce_static(h, ctypes.byref(d))
    if code != PLBM_OK and not (allow_unstable and code == PLBM_E_UNSTABLE):
        check(code)
    return d


def plbm_destroy(h):
    if h:
        load().plbm_destroy(h)


def plbm_batch_bytes(max_slots, max_tiles):
    n = _U64()
    check(load().plbm_batch_bytes(max_slots, max_tiles, ctypes.byref(n)))
    return n.value


def plbm_batch_create(max_slots, max_tiles, dev_ptr, dev_bytes, stream_ptr):
    h = _VP()
    check(load().plbm_batch_create(max_slots, max_tiles, dev_ptr, dev_bytes, stream_ptr, ctypes.byref(h)))
    return h.value


def plbm_batch_attach(b, lat):
    s = _I32()
    check(load().plbm_batch_attach(b, lat, ctypes.byref(s)))
    return s.value


def plbm_batch_detach(b, slot):
    check(load().plbm_batch_detach(b, slot))


def plbm_batch_step(b, n):
    check(load().plbm_batch_step(b, int(n)))


def plbm_batch_diag(b, max_slots):
    arr = (plbm_diag * max_slots)()
    check(load().plbm_batch_diag(b, arr))
    return list(arr)


def plbm_batch_destroy(b):
    if b:
        load().plbm_batch_destroy(b)
