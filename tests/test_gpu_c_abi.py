"""The C ABI used from plain C on the GPU: tests/c/abi_smoke.c, compiled with the
host C compiler against include/plbm.h and linked to the in-tree libplbm.so and
the HIP runtime, creates a lattice on its own hipMalloc buffer and the legacy
null stream, steps it, and checks health flags, exact mass conservation and the
undersized-buffer error (no Python or PyTorch in the process)."""
import os
import shutil
import subprocess

import pytest

from gpu_cases import fmt, require_gpu

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_plain_c_program_drives_the_library(tmp_path):
    require_gpu()
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lib_dir = os.path.join(ROOT, "paper_2504_15018_amd")
    assert os.path.exists(os.path.join(lib_dir, "libplbm.so")), "libplbm.so is not built"
    exe = tmp_path / "abi_smoke"
    subprocess.run([cc, "-std=c11", "-O2", "-D__HIP_PLATFORM_AMD__", f"-I{ROOT}/include", f"-I{ROCM}/include",
                    os.path.join(ROOT, "tests", "c", "abi_smoke.c"), "-o", str(exe), f"-L{lib_dir}", "-lplbm",
                    f"-L{ROCM}/lib", "-lamdhip64", "-lm", f"-Wl,-rpath,{lib_dir}", f"-Wl,-rpath,{ROCM}/lib"],
                   check=True)
    fmt("c_abi_run")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("c_abi t=40 ")
