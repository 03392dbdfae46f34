"""Build libplbm.so for gfx950 in-tree (hipcc, no JIT cache).

Usage: python -m paper_2504_15018_amd.build [--jobs N]
Each population-storage kernel file is its own translation unit; the float64
one is compiled without floating-point contraction so that its rounding
follows the plain operation order.
"""
import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libplbm.so")

ARCH = "gfx950"
COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions are generated
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]
SOURCES = {
    # Per storage, the kernel shape measured fastest on MI355X (256^3 D3Q19
    # BGK/MRT, 384x384x128 channel): the halo ring on waves of its own (with
    # issue priority) and tiles 64 nodes wide (the x-halo columns read lines
    # that only the neighbouring tile otherwise uses, so fewer columns per
    # node pay most); float32 and the 16-bit formats 64 x 8 tiles (eleven
    # waves, three per SIMD, one workgroup per CU), the globally shifted 16-bit
    # formats with loads a full plane iteration ahead, the others one phase
    # ahead (the locally shifted ones run 17 % slower a full plane ahead); float64 64 x 4 tiles
    # (seven waves within 256 registers).  Populations are stored with the
    # non-temporal hint.  The in-place pattern's kernels (no halo waves) use
    # 64 x 4 tiles in 16-bit storage: three workgroups of four waves per CU
    # instead of one of eight hide the latency of these instruction-bound
    # formats (256^3 step 0.787 -> 0.640 ms in f16r, 0.660 -> 0.540 in bf16s;
    # 64 x 12 and 32 x 4 were slower); float32 stays fastest at 64 x 8, and so
    # does float64 (two workgroups of four waves at 220 registers; 256^3 step
    # 1.665 -> 1.559 ms; 32 x 8 1.700).
    "plbm_k_f64.hip": ["-ffp-contract=off", "-DPLBM_PREFETCH=1", "-DPLBM_D3_TX=64", "-DPLBM_D3_TY=4", "-DPLBM_AA_TY=8"],
    "plbm_k_f32.hip": ["-DPLBM_PREFETCH=1", "-DPLBM_D3_TX=64", "-DPLBM_D3_TY=8", "-DPLBM_MIN_WAVES=3"],
    "plbm_k_f16s.hip": ["-DPLBM_PREFETCH=2", "-DPLBM_D3_TX=64", "-DPLBM_D3_TY=8", "-DPLBM_MIN_WAVES=3", "-DPLBM_AA_TY=4"],
    "plbm_k_bf16s.hip": ["-DPLBM_PREFETCH=2", "-DPLBM_D3_TX=64", "-DPLBM_D3_TY=8", "-DPLBM_MIN_WAVES=3", "-DPLBM_AA_TY=4"],
    "plbm_k_f16r.hip": ["-DPLBM_PREFETCH=1", "-DPLBM_D3_TX=64", "-DPLBM_D3_TY=8", "-DPLBM_MIN_WAVES=3", "-DPLBM_AA_TY=4"],
    "plbm_k_bf16r.hip": ["-DPLBM_PREFETCH=1", "-DPLBM_D3_TX=64", "-DPLBM_D3_TY=8", "-DPLBM_MIN_WAVES=3", "-DPLBM_AA_TY=4"],
    "plbm_api.hip": [],
    "plbm_params.cpp": ["-x", "hip", "-ffp-contract=off"],
}


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src, extra):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    return obj


def build(jobs=None, verbose=False, out=None, defines=()):
    """Compile every source and link libplbm.so (or `out`)."""
    global BUILD
    if out is not None:
        BUILD = os.path.join(os.path.dirname(os.path.abspath(out)), "_build")
    os.makedirs(BUILD, exist_ok=True)
    extra_defs = [f"-D{d}" for d in defines]
    jobs = jobs or min(6, os.cpu_count() or 2)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda kv: _compile(kv[0], kv[1] + extra_defs), SOURCES.items()))
    lib = os.path.abspath(out) if out is not None else LIB
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


# Host-side sanitizer build: the host layer (plbm_api.hip, plbm_params.cpp)
# with AddressSanitizer and UndefinedBehaviorSanitizer on the host pass only
# (each -fsanitize= follows -Xarch_host; device code is unchanged), linked
# with the kernel objects of the regular build into _san/libplbm.so.  Load it
# with PLBM_LIB and the ASan runtime preloaded (sanitizer_runtime()).
SAN_DIR = os.path.join(PKG, "_san")
SAN_LIB = os.path.join(SAN_DIR, "libplbm.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
HOST_SOURCES = ("plbm_api.hip", "plbm_params.cpp")


def sanitizer_runtime():
    """Path of the compiler's shared ASan runtime (to preload into a non-instrumented host process)."""
    r = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(p) or not os.path.exists(p):
        raise RuntimeError("ASan runtime not found")
    return p


def build_sanitized(verbose=False):
    """Build _san/libplbm.so: sanitized host layer + the regular kernel objects (build() first)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    kernel_objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in SOURCES if s not in HOST_SOURCES]
    missing = [o for o in kernel_objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"kernel objects missing ({missing[0]}): run build() first")
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(SAN_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc()] + COMMON + SOURCES[src] + SAN_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
        objs.append(obj)
    tmp = SAN_LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan", "-Xarch_host",
           "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o", tmp] + objs + kernel_objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, SAN_LIB)
    if verbose:
        print(f"built {SAN_LIB}")
    return SAN_LIB


PROBE_SRC = "probe_stream.hip"
PROBE_LIB = os.path.join(PKG, "libplbm_probe.so")


def build_probe(verbose=False):
    """Compile the bandwidth probes (the benchmark's reference points) into libplbm_probe.so."""
    tmp = PROBE_LIB + ".tmp"
    cmd = [hipcc()] + COMMON + ["-shared", os.path.join(CSRC, PROBE_SRC), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, PROBE_LIB)
    if verbose:
        print(f"built {PROBE_LIB}")
    return PROBE_LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--out", default=None, help="library path (default: in-tree libplbm.so)")
    ap.add_argument("-D", dest="defines", action="append", default=[], help="extra preprocessor definition")
    a = ap.parse_args()
    build(a.jobs, verbose=True, out=a.out, defines=a.defines)
    if a.out is None:
        build_probe(verbose=True)
    sys.exit(0)
