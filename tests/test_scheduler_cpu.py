"""The serving scheduler's host-only parts (csrc/sched.hpp: arena, percentile
rule, admission pass) against a fake executor and clock, on the CPU: a
discrete-event simulation compiled with g++ (tests/cpp/sched_sim.cpp).

Checked: arena ranges never overlap, its accounting is exact and freeing
everything coalesces; nearest-rank percentiles; near saturation the memory
and slot limits hold at every step, a request only overtakes older ones that
were offered in the same pass and did not fit, and every request completes;
a large request behind a steady stream of small ones is admitted after a
bounded number of passes, and with that rule switched off only once the
stream stops; the default size-aware order (aged requests first, then by
modelled cost) with at most one large request in flight keeps its order,
its cap and the limits, completes every request within the aging bound
plus a few large services, and cuts the small requests' mean wait below
that of arrival order.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# Plain build, AddressSanitizer + UndefinedBehaviorSanitizer (out-of-bounds,
# use-after-free and leaks in the arena's bookkeeping, integer overflow in
# the size arithmetic), and ThreadSanitizer (the simulation is single
# threaded: the build keeps the headers clean of anything that would race
# once a second thread uses them).
SANITIZERS = {
    "plain": [],
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"],
    "tsan": ["-fsanitize=thread", "-g"],
}


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("flavour", list(SANITIZERS))
def test_scheduler_simulation(tmp_path, flavour):
    exe = tmp_path / "sched_sim"
    src = os.path.join(ROOT, "tests", "cpp", "sched_sim.cpp")
    inc = os.path.join(ROOT, "paper_1811_07325_amd", "csrc")
    build = subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror"] + SANITIZERS[flavour] +
                           ["-I", inc, src, "-o", str(exe)], capture_output=True, text=True)
    if build.returncode != 0 and flavour != "plain" and "cannot find" in build.stderr:
        pytest.skip(f"{flavour} runtime not installed: {build.stderr.strip()[:200]}")
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "all ok" in run.stdout
    assert "Sanitizer" not in run.stderr, run.stderr
