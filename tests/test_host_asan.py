"""The C ABI's host code under AddressSanitizer: the library built with the
host part instrumented (device code as usual) passes the argument-checking
tests of test_abi_cpu.py, run in a child process with the sanitizer runtime
preloaded.  No GPU is used: the argument-checking context touches no device."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_checks_under_address_sanitizer():
    from paper_1804_06231_amd import build
    rt = build.asan_runtime()
    if not rt:
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    lib = build.build_asan(jobs=8)
    env = dict(os.environ, LD_PRELOAD=rt, PVL_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
