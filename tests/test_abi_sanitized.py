"""The ABI tests of tests/test_abi.py (no GPU) run against the library's host
code built with AddressSanitizer and UndefinedBehaviorSanitizer
(``paper_2306_05332_amd.build_sanitized``): argument validation,
the hierarchy and App. A.3 host arithmetic, tuning-table round trips and the
error paths, in a child process with the clang ASan runtime preloaded.  Any
sanitizer report fails the test.  The build takes about two minutes and is
reused while no source is newer than it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale(lib, dirs):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    for d in dirs:
        for name in os.listdir(d):
            if name.endswith((".hip", ".h", ".py")) and os.path.getmtime(os.path.join(d, name)) > t:
                return True
    return False


def test_abi_under_host_sanitizers():
    sys.path.insert(0, ROOT)
    from paper_2306_05332_amd import build_sanitized as B
    try:
        asan = B.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    lib = B.HOST_SAN_LIB
    if _stale(lib, [B.CSRC, B.INCLUDE, B.PKG]):
        B.build_host_sanitized()
    # the library is instrumented (it calls into the ASan and UBSan runtimes)
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms
    env = dict(os.environ, RKL_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       env=env, capture_output=True, text=True, cwd=ROOT, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
