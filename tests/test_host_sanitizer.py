"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer: every source
file is compiled with the sanitizers on its host side and linked with tests/host_check.cpp, a
driver of host-only checks (configuration validation and level planning for every family of
configurations, entry-point argument checks, the reference element and Gauss rule at every
order, the dense SPD inverse, the tridiagonal eigenvalue). No GPU call is made."""

import os
import shutil
import subprocess

import pytest

from paper_1402_5938_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(not os.path.exists(build.HIPCC), reason="hipcc not installed")
def test_host_code_under_sanitizers(tmp_path):
    exe = build.build_host_check(os.path.join(HERE, "host_check.cpp"), str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "host checks: ok" in r.stdout
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    shutil.rmtree(tmp_path, ignore_errors=True)
