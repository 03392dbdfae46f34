"""Host logic of bench.py (no GPU): the one-GPU contract, the identity of the
profiled kernel, and which workloads may report profiled HBM traffic."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_hash_ignores_include_paths_but_not_flags(monkeypatch):
    import bench
    from paper_2504_15018_amd import build
    h0 = bench.kernel_source_hash()
    moved = [("-I/elsewhere" + a[2:]) if a.startswith("-I") else a for a in build.COMMON]
    monkeypatch.setattr(build, "COMMON", moved)
    assert bench.kernel_source_hash() == h0  # another checkout of the same sources
    flags = dict(build.SOURCES)
    flags["plbm_k_f32.hip"] = flags["plbm_k_f32.hip"] + ["-DPLBM_PREFETCH=2"]
    monkeypatch.setattr(build, "SOURCES", flags)
    assert bench.kernel_source_hash() != h0  # another kernel


def test_profiled_traffic_only_for_the_profiled_workload():
    import bench
    assert bench.profiled_traffic("f16r", "mrt", 256) is None
    assert bench.profiled_traffic("f32", "bgk", 256) is None
    assert bench.profiled_traffic("f32", "mrt", 128) is None
    t = bench.profiled_traffic("f32", "mrt", 256)
    assert t is None or 2.0e9 < t < 4.0e9  # bytes per update launch when the profile matches the sources


def test_probe_library_exports_its_two_probes():
    import ctypes
    path = os.path.join(ROOT, "paper_2504_15018_amd", "libplbm_probe.so")
    if not os.path.exists(path):
        import pytest
        pytest.skip("libplbm_probe.so not built")
    lib = ctypes.CDLL(path)
    assert hasattr(lib, "plbm_probe_stream19") and hasattr(lib, "plbm_probe_copy4")
