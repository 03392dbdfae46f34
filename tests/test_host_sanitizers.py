"""The library's host layer (C ABI entry points, layout, parameter resolution:
plbm_api.hip and plbm_params.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

The sanitized library (build.build_sanitized: host pass instrumented, device
code unchanged, linked with the regular kernel objects) is loaded through
PLBM_LIB into a child process with the ASan runtime preloaded, which runs
the CPU ABI tests (tests/test_abi.py: exports, struct layouts, parameter
chain against the oracle, error paths, size limits; no kernel launches).  Any
sanitizer report fails the child (UBSan does not recover).
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_tests_pass_under_asan_and_ubsan():
    from paper_2504_15018_amd import build as B

    if not all(os.path.exists(os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o")) for s in B.SOURCES):
        B.build()
    lib = B.build_sanitized()
    env = dict(os.environ)
    env.update({
        "PLBM_LIB": lib,
        "LD_PRELOAD": B.sanitizer_runtime(),
        # the interpreter itself is not instrumented: no leak report for it, no link-order check
        "ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:detect_odr_violation=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
    })
    probe = subprocess.run([sys.executable, "-c", "import sys; sys.path.insert(0, %r); "
                            "from paper_2504_15018_amd import native as N; N.load(); print(N._lib._name)" % ROOT],
                           env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0, probe.stderr[-3000:]
    assert probe.stdout.strip().splitlines()[-1] == lib
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi.py")], env=env, capture_output=True, text=True,
                       timeout=900, cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
