"""Admission policy of the serving loop (host logic, no GPU): a C++ driver runs
the policy header the library uses against a mock device backend and a
simulated clock, and checks that the budget and the slot limits always hold,
that requests are admitted in arrival order and all complete, that pooled
hierarchies are reused and released only when the budget or the device needs
it, and that device errors are reported."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_admission_policy(tmp_path):
    exe = tmp_path / "sched_check"
    src = os.path.join(ROOT, "tests", "sched_check.cpp")
    inc = os.path.join(ROOT, "paper_1406_5369_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", f"-I{inc}", src, "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    lines = out.stdout.strip().splitlines()
    assert [ln.split(":")[0] for ln in lines] == ["ok cases", "ok roomy", "ok tight_budget", "ok device_oom",
                                                  "ok one_slot"]
