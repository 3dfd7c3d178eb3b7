"""Sanitizer runs of the host code (CPU; no GPU needed):

* the Gram-Schmidt admission budget (group_budget.h) under AddressSanitizer + UBSan and
  under ThreadSanitizer (16 threads acquiring and releasing);
* the oracle's C projectors (oracle/projectors.c) under AddressSanitizer + UBSan on small
  ragged geometries, with the adjoint identities checked;
* the library with its host code instrumented (paper_2110_01481_amd/build.py
  build_host_sanitized: -Xarch_host before every -fsanitize=, device code as usual) driven
  by an instrumented C++ program through every C-ABI entry point: invalid arguments here;
  with a GPU the same program also runs solves of every kind (test_gpu_sanitized_host).
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2110_01481_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, env=ENV, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0 and r.stdout.strip().splitlines()[-1] == "ok", r.stdout + r.stderr


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_group_budget_under_sanitizers(tmp_path, san):
    exe = tmp_path / "gb"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", f"-fsanitize={san}",
                    "-fno-omit-frame-pointer", "-I", CSRC,
                    os.path.join(NATIVE, "group_budget_check.cpp"), "-o", str(exe)], check=True)
    _run([str(exe)])


def test_oracle_projectors_under_sanitizers(tmp_path):
    exe = tmp_path / "osc"
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-fopenmp", "-I",
                    os.path.join(ROOT, "oracle"), os.path.join(NATIVE, "oracle_sanitize_check.c"),
                    "-o", str(exe), "-lm"], check=True)
    _run([str(exe)], env=dict(ENV, OMP_NUM_THREADS="4"))


def sanitized_check_program():
    """Builds the host-instrumented library and the check program (in-tree, under
    paper_2110_01481_amd/_san/) and returns the program's path."""
    from paper_2110_01481_amd.build import SANITIZED_LIB, build_host_sanitized
    build_host_sanitized()
    exe = os.path.join(os.path.dirname(SANITIZED_LIB), "capi_sanitize_check")
    subprocess.run([CLANG, "-std=c++17", "-O1", "-g", "-Wno-unused-result", "-Wno-unused-value",
                    "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I",
                    os.path.join(ROOT, "include"), os.path.join(NATIVE, "capi_sanitize_check.cpp"),
                    "-o", exe, SANITIZED_LIB, "-L", "/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib", "-Wl,-rpath,$ORIGIN"], check=True)
    return exe


def test_capi_host_code_under_sanitizers():
    # the HIP runtime's own allocations at exit are not the library's: no leak check
    _run([sanitized_check_program()], env=dict(ENV, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1"))
