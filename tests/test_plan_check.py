"""The work-item planner checked on the host: compile tests/plan_check.cpp
(the library's host code with the kernel launchers stubbed out) and run it
over named shapes and random batches of every kind."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
def test_planner_bounds_and_races(tmp_path):
    exe = tmp_path / "plan_check"
    cmd = ["g++", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
           "-D__HIP_PLATFORM_AMD__", "-o", str(exe), os.path.join(HERE, "plan_check.cpp"),
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    tail = run.stdout.strip().splitlines()[-3:]
    assert run.returncode == 0 and tail[-1] == "bad 0", "\n".join(tail)
    assert "fuzz runs 400" in run.stdout
