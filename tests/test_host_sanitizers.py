"""Host-only sources of libtucker (the TTM-tree planner, Sec. 3, and the
processor-grid planner, Sec. 4) built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer, and driven through the C ABI by
tests/host_sanitize_driver.cpp: seeded shapes of 2 to 10 modes and the widest
supported count, every tree kind, k-best plans, string and node buffers of
exact and short sizes, static and dynamic grids, and invalid arguments.  Any
sanitizer report or failed check fails the test.  CPU only; skipped where g++
or the sanitizer runtimes are missing."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_05594_amd", "csrc")


def test_planner_and_grids_clean_under_asan_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "grid.cpp"),
           os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in (r.stderr or "").lower():
        pytest.skip(f"sanitizer runtimes unavailable: {r.stderr[-300:]}")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "host driver ok" in run.stdout
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr
