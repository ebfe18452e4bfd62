"""AddressSanitizer / UndefinedBehaviorSanitizer build of the host-side
nested-dissection planner (CPU only).

nd_plan.cpp is plain host C++ (it builds the coarse solver's front tree and
index maps); it is compiled here with the host compiler, without any device
code, together with tests/sanitize/nd_plan_driver.cpp, and run on the coarse
grids of the configurations: the benchmark's 513 x 513 reach-2 plan, the
batching workload's reach-3 plans, rectangular and degenerate grids.  Any
out-of-bounds access, leak or undefined behaviour aborts the driver.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_03571_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "nd_plan_driver.cpp")


def compiler():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++") or ""):
        if c and os.path.exists(c):
            return c
    pytest.skip("no clang++ with the sanitizer runtimes")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("san") / "nd_plan_driver")
    cmd = [compiler(), "-x", "c++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", CSRC,
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(CSRC, "nd_plan.cpp"), DRIVER, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def run(driver, quads):
    args = [str(v) for q in quads for v in q]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, *args], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_planner_checked_grids_under_sanitizers(driver):
    # ncx, ncy, reach, leaf, check: structural check (every node eliminated
    # once, every boundary the exact Schur support) on grids it finishes fast
    out = run(driver, [(9, 9, 2, 8, 1), (33, 17, 3, 8, 1), (129, 129, 2, 8, 1), (5, 40, 1, 3, 1),
                       (1, 1, 2, 8, 1), (63, 63, 3, 8, 1), (31, 31, 1, 8, 1)])
    assert out.count("status 0") == 7


def test_planner_full_size_grids_under_sanitizers(driver):
    # the benchmark's coarse grid (513^2, reach 2) and the batching
    # workload's largest (129^2, reach 3), planned without the O(N * fronts) check
    out = run(driver, [(513, 513, 2, 8, 0), (129, 129, 3, 8, 0), (257, 1, 2, 8, 0)])
    assert out.count("plan ") == 3
