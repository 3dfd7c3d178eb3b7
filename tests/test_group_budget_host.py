"""Host-side admission of spinning Gram-Schmidt block groups (GroupBudget in
paper_2110_01481_amd/csrc/group_budget.h): unit arithmetic, waiting, arrival order and
the capacity invariant under 16 threads. The checks are C++ (tests/native), built with
g++ and run here; the header holds no HIP code."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_group_budget_checks(tmp_path):
    exe = tmp_path / "group_budget_check"
    src = os.path.join(ROOT, "tests", "native", "group_budget_check.cpp")
    inc = os.path.join(ROOT, "paper_2110_01481_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-pthread", "-Wall", "-Werror", "-I", inc, src,
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
