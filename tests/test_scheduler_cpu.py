"""The serving scheduler's host-only parts (csrc/sched.hpp: arena, percentile
rule, admission pass) against a fake executor and clock, on the CPU: a
discrete-event simulation compiled with g++ (tests/cpp/sched_sim.cpp).

Checked: arena ranges never overlap, its accounting is exact and freeing
everything coalesces; nearest-rank percentiles; near saturation the memory
and slot limits hold at every step, a request only overtakes older ones that
were offered in the same pass and did not fit, and every request completes;
a large request behind a steady stream of small ones is admitted after a
bounded number of passes, and with that rule switched off only once the
stream stops.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scheduler_simulation(tmp_path):
    exe = tmp_path / "sched_sim"
    src = os.path.join(ROOT, "tests", "cpp", "sched_sim.cpp")
    inc = os.path.join(ROOT, "paper_1811_07325_amd", "csrc")
    build = subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror", "-I", inc, src, "-o", str(exe)],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "all ok" in run.stdout
