"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU, no GPU): the serving scheduler in simulate mode (both modes, worker and
manual stepping, with and without a token limit) and the C ABI's argument
validation, driven by tests/host_check/host_check.cpp."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "host_check"))


@pytest.mark.timeout(900)
def test_host_code_clean_under_asan_and_ubsan():
    import build as host_build
    exe = host_build.build()
    env = dict(os.environ)
    # leaks inside the ROCm runtime at exit are not this library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["HIP_VISIBLE_DEVICES"] = env.get("HIP_VISIBLE_DEVICES", "")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "host checks passed" in r.stdout
