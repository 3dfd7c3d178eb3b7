"""The library's host code under AddressSanitizer and UBSan on a GPU: the instrumented
check program (tests/native/capi_sanitize_check.cpp, built with the host-instrumented
library by tests/test_sanitizers_host.py into paper_2110_01481_amd/_san/) runs small
solves of every kind through the C ABI -- AB/BA-GMRES under each stop rule and precision,
error histories, LSQR/LSMR, an engine with continuous admission, the projectors, the
allocation-free forward projection, launch timing -- and releases everything; the
sanitizers abort on any heap error or undefined behaviour in the host code."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2110_01481_amd", "_san", "capi_sanitize_check")


def test_capi_host_code_under_sanitizers_on_gpu():
    if not os.path.exists(EXE):
        pytest.skip("sanitized check program not built (tests/test_sanitizers_host.py builds it)")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and r.stdout.strip().splitlines()[-1] == "ok"
