"""The library's host code (plan building, argument checks, the solver's and
the out-of-core driver's host logic) under AddressSanitizer and
UndefinedBehaviorSanitizer on the CPU: the ABI checks of test_abi_cpu.py run
in a child process against the sanitized build, with the ASan runtime
preloaded, and must pass with no sanitizer report.  (No GPU code is
sanitized: each -fsanitize= of that build applies to the host only.)"""
import os
import subprocess
import sys

import pytest

from paper_1809_09725_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(B.asan_runtime() is None, reason="no clang ASan runtime in this image")
def test_abi_checks_under_host_sanitizers():
    lib = B.build_sanitized()
    env = dict(os.environ, LD_PRELOAD=B.asan_runtime(), RT4D_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join("tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
    assert " passed" in r.stdout
