"""Host-only check (no GPU) that no render launch asks for more LDS than one
workgroup may allocate, for every launch shape and residency setting: the
arithmetic of csrc/launch_budget.hpp compiled on its own with g++."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2208_12737_amd", "csrc")


def test_lds_requests_fit_one_workgroup(tmp_path):
    exe = str(tmp_path / "launch_budget_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC, "-o", exe,
                    os.path.join(HERE, "c", "launch_budget_check.cpp")], check=True)
    res = subprocess.run([exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok"), res.stdout
