"""CPU checks of the C-ABI library: it loads, exports every entry point the
header declares, and its host parameter layer (eqs. unit, unit2, thickness,
surface_tension and the mechanical-stability coexistence) agrees with the
oracle.  No kernel is launched here.
"""
import ctypes
import json
import os
import re

import numpy as np
import pytest

from oracle import eos as E
from oracle import params as P
from paper_2504_15018_amd import native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))


def _declared():
    src = open(os.path.join(ROOT, "include", "plbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(plbm_[a-z0-9_]+)\s*\(", src)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = N.load()
    names = _declared()
    assert len(names) == len(N.EXPORTED) == 25
    for n in names:
        assert hasattr(lib, n), n
        assert n in N.EXPORTED, n
    assert N.plbm_abi_version() == N.PLBM_ABI_VERSION


def test_struct_layouts_match_the_header(tmp_path):
    """Compile the header with the host C compiler and compare every field offset."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = [N.plbm_phys_params, N.plbm_lattice_map, N.plbm_lattice_params, N.plbm_lattice_desc,
               N.plbm_shape, N.plbm_diag]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "plbm.h"', "int main(void) {"]
    expect = []
    for st in structs:
        n = st.__name__
        lines.append(f'printf("%zu\\n", sizeof({n}));')
        expect.append(ctypes.sizeof(st))
        for fname, _ in st._fields_:
            lines.append(f'printf("%zu\\n", offsetof({n}, {fname}));')
            expect.append(getattr(st, fname).offset)
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == expect


def _phys_paper(gamma=7.58e-3, xi=1.5e-7, L=10e-6, bf=(0.0, 0.0, 0.0)):
    t = GOLD["table_I_R134a_30C"]
    ph = N.plbm_phys_params()
    ph.eos = N.PLBM_EOS_PAPER
    ph.rho_v, ph.rho_l = t["rho_v_kg_m3"], t["rho_l_kg_m3"]
    ph.nu_v, ph.nu_l = t["nu_v_mm2_s"] * 1e-6, t["nu_l_mm2_s"] * 1e-6
    ph.gamma, ph.xi, ph.L = gamma, xi, L
    for a in range(3):
        ph.body_force[a] = bf[a]
    return ph


def test_resolve_params_matches_oracle_chain():
    fluid = P.R134A_30C
    for Nx, xi, tau, gam in [(100, 1.5, 0.56, 7.58e-3), (200, 3.0, 0.68, 0.758e-3), (500, 7.5, 0.52, 75.8e-3)]:
        m = N.plbm_lattice_map()
        m.L_lat, m.tau_l, m.rho_l_lat = Nx, tau, 1.187
        out = N.plbm_resolve_params(_phys_paper(gamma=gam, xi=xi * 10e-6 / Nx, bf=(1e6, 0, 0)), m)
        ref = P.resolve_paper(fluid, 10e-6, Nx, xi, tau_l=tau, gamma=gam, body_force=(1e6, 0, 0))
        for a, b in [(out.C_L, ref.conv.C_L), (out.C_T, ref.conv.C_T), (out.C_M, ref.conv.C_M),
                     (out.C_U, ref.conv.C_U), (out.C_VF, ref.conv.C_VF), (out.C_gamma, ref.conv.C_gamma),
                     (out.K, ref.K), (out.kappa, ref.kappa), (out.tau_v, ref.tau_v),
                     (out.eos_rho_v, ref.rho_v), (out.body_force[0], ref.Fg[0])]:
            assert a == pytest.approx(b, rel=1e-13)
        # predicted coexistence at finite psi (quadrature-limited agreement)
        e = E.PaperEOS(ref.K, ref.rho_v, ref.rho_l)
        cv, cl, _ = P.coexistence(e, 2.0, rho_hi=3.0 * ref.rho_l)
        assert out.rho_v == pytest.approx(cv, rel=1e-9) and out.rho_l == pytest.approx(cl, rel=1e-11)


@pytest.mark.parametrize("tr", [0.6, 0.7, 0.8, 0.9])
def test_pr_lattice_params_match_oracle(tr):
    out = N.plbm_params_pr_lattice(tr, 0.326, 2.0, 1.0, 1.0, 1.0)
    e = E.PengRobinsonEOS(tr, 0.326)
    cv, cl, _ = P.coexistence(e, 2.0)
    assert out.pr_T == pytest.approx(e.T, rel=1e-15)
    assert out.pr_alpha == pytest.approx(e.alpha, rel=1e-15)
    assert out.rho_v == pytest.approx(cv, rel=1e-9) and out.rho_l == pytest.approx(cl, rel=1e-11)


def test_pr_surface_tension_mapping_matches_oracle():
    ph = N.plbm_phys_params()
    ph.eos = N.PLBM_EOS_PENG_ROBINSON
    ph.rho_v, ph.rho_l, ph.nu_v, ph.nu_l = 37.5, 1187.0, 0.339e-6, 0.158e-6
    ph.gamma, ph.L, ph.T_over_Tc, ph.omega = 7.58e-3, 10e-6, 0.8, 0.326
    m = N.plbm_lattice_map()
    m.L_lat, m.tau_l, m.rho_l_lat = 100, 0.56, 0.0
    out = N.plbm_resolve_params(ph, m)
    e = E.PengRobinsonEOS(0.8, 0.326)
    cv, cl, p0 = P.coexistence(e, 2.0)
    gk = P.gamma_over_kappa_general(e, cv, cl, p0)
    assert out.gamma_lat / out.kappa == pytest.approx(gk, rel=2e-6)


def test_invalid_arguments_are_reported():
    with pytest.raises(N.PlbmError) as ei:
        N.plbm_params_pr_lattice(1.2)
    assert ei.value.code == N.PLBM_E_INVALID
    with pytest.raises(N.PlbmError) as ei:
        N.plbm_params_paper_lattice(1.0, 0.5, 3.0)
    assert ei.value.code == N.PLBM_E_INVALID
    assert "rho" in N.plbm_last_error()
    m = N.plbm_lattice_map()
    m.L_lat, m.tau_l = 100, 0.4
    with pytest.raises(N.PlbmError):
        N.plbm_resolve_params(_phys_paper(), m)


def test_lattice_bytes_and_validation():
    from paper_2504_15018_amd.lattice import make_desc
    d = make_desc("D3Q19", (64, 48, 40), storage="f32")
    nb = N.plbm_lattice_bytes(d)
    n = 64 * 48 * 40
    assert nb >= 2 * 19 * n * 4 + 4 * n * 8 + 3 * n * 4
    assert nb < 2 * 19 * n * 4 + 4 * n * 8 + 3 * n * 4 + 4 << 20
    d16 = make_desc("D3Q19", (64, 48, 40), storage="f16s")
    assert N.plbm_lattice_bytes(d16) < nb
    bad = make_desc("D2Q9", (8, 8))
    bad.nz = 3
    with pytest.raises(N.PlbmError) as ei:
        N.plbm_lattice_bytes(bad)
    assert ei.value.code == N.PLBM_E_INVALID
    walls_x = make_desc("D3Q19", (8, 8, 8))
    walls_x.bc[0] = N.PLBM_HALFWAY_BB
    with pytest.raises(N.PlbmError) as ei:
        N.plbm_lattice_bytes(walls_x)
    assert ei.value.code == N.PLBM_E_UNSUPPORTED


def test_inplace_pattern_bytes_and_validation():
    """The in-place pattern holds one population array plus a psi array."""
    from paper_2504_15018_amd.lattice import make_desc
    n = 64 * 48 * 40
    for st, S, C in (("f32", 4, 4), ("f64", 8, 8), ("bf16s", 2, 4)):
        ab = N.plbm_lattice_bytes(make_desc("D3Q19", (64, 48, 40), storage=st))
        aa = N.plbm_lattice_bytes(make_desc("D3Q19", (64, 48, 40), storage=st, pattern="aa"))
        saved = ab - aa
        # one population array less (with a trash area of at most 40 KiB per
        # z plane for ragged-tile lanes), one psi array more
        assert 19 * n * S - n * C <= saved <= 19 * n * S - n * C + 40 * 40 * 1024 + (1 << 20)
    for st in ("f16r", "bf16r"):  # one population array; the two reference-density arrays stay
        ab = N.plbm_lattice_bytes(make_desc("D3Q19", (64, 48, 40), storage=st))
        aa = N.plbm_lattice_bytes(make_desc("D3Q19", (64, 48, 40), storage=st, pattern="aa"))
        assert 19 * n * 2 - n * 4 <= ab - aa <= 19 * n * 2 - n * 4 + 40 * 40 * 1024 + (1 << 20)
    bad = make_desc("D2Q9", (8, 8))
    bad.pattern = 7
    with pytest.raises(N.PlbmError) as ei:
        N.plbm_lattice_bytes(bad)
    assert ei.value.code == N.PLBM_E_INVALID


def test_size_limits():
    """At most 2^31 - 1 nodes (32-bit node indices in the kernels) and 2 GiB of
    populations per z plane (32-bit byte offsets within a plane)."""
    from paper_2504_15018_amd.lattice import make_desc
    assert N.plbm_lattice_bytes(make_desc("D3Q19", (1290, 1290, 1290), storage="f16s", pattern="aa")) > 0
    with pytest.raises(N.PlbmError) as ei:
        N.plbm_lattice_bytes(make_desc("D3Q19", (1291, 1291, 1291), storage="f16s"))
    assert ei.value.code == N.PLBM_E_INVALID
    # D2Q9 kernel planes are single rows: 2^26 nodes of float64 are 4.8 GB
    with pytest.raises(N.PlbmError) as ei:
        N.plbm_lattice_bytes(make_desc("D2Q9", (1 << 26, 4), storage="f64"))
    assert ei.value.code == N.PLBM_E_UNSUPPORTED
    assert N.plbm_lattice_bytes(make_desc("D2Q9", (1 << 22, 4), storage="f64")) > 0


def test_wall_density_validation():
    from paper_2504_15018_amd.lattice import make_desc
    ok = make_desc("D3Q19", (16, 16, 16), walls=True, rho_wall=(6.0, 0.0))
    assert N.plbm_lattice_bytes(ok) == N.plbm_lattice_bytes(make_desc("D3Q19", (16, 16, 16), walls=True))
    for bad in (make_desc("D3Q19", (16, 16, 16), rho_wall=(6.0, 0.0)),  # no walls
                make_desc("D2Q9", (16, 16), walls=True, rho_wall=(-1.0, 0.0)),
                make_desc("D2Q9", (16, 16), walls=True, rho_wall=(0.0, float("nan")))):
        with pytest.raises(N.PlbmError) as ei:
            N.plbm_lattice_bytes(bad)
        assert ei.value.code == N.PLBM_E_INVALID


def test_create_rejects_small_buffer_before_touching_the_device():
    from paper_2504_15018_amd.lattice import make_desc
    d = make_desc("D2Q9", (16, 16))
    p = N.plbm_params_pr_lattice(0.8)
    nb = N.plbm_lattice_bytes(d)
    with pytest.raises(N.PlbmError) as ei:
        N.plbm_create(d, p, 4096, nb - 1, None)  # a fake, aligned address: never dereferenced
    assert ei.value.code == N.PLBM_E_NOMEM
    with pytest.raises(N.PlbmError) as ei:
        N.plbm_create(d, p, 4096 + 8, nb, None)
    assert ei.value.code == N.PLBM_E_INVALID


def test_well_balanced_scheme_validation():
    """The well-balanced scheme: its extra per-node array is counted; unsupported combinations and a
    non-positive gradient coefficient are refused (no kernel runs)."""
    from paper_2504_15018_amd.lattice import make_desc
    base = N.plbm_lattice_bytes(make_desc("D3Q19", (40, 24, 18), storage="f32"))
    wb = N.plbm_lattice_bytes(make_desc("D3Q19", (40, 24, 18), storage="f32", wb_k=0.15))
    assert wb - base >= 40 * 24 * 18 * 4  # the chemical potential, float32
    for kw in ({"storage": "f16r"}, {"storage": "bf16s"}, {"pattern": "aa"}, {"walls": True, "rho_wall": (0.5, 0.0)}):
        with pytest.raises(N.PlbmError) as e:
            N.plbm_lattice_bytes(make_desc("D2Q9", (16, 16), wb_k=0.15, **kw))
        assert e.value.code == N.PLBM_E_UNSUPPORTED, kw
    d = make_desc("D2Q9", (16, 16))
    d.scheme = N.PLBM_SCHEME_WELL_BALANCED
    d.wb_k = -1.0
    with pytest.raises(N.PlbmError) as e:
        N.plbm_lattice_bytes(d)
    assert e.value.code == N.PLBM_E_INVALID
    d.scheme = 7
    with pytest.raises(N.PlbmError) as e:
        N.plbm_lattice_bytes(d)
    assert e.value.code == N.PLBM_E_INVALID
