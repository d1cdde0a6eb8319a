"""The serving scheduler's logic on the CPU, under the sanitizers.

tests/cpu/scheduler_fake_exec.cpp drives the device-independent scheduler
(paper_2503_22652_amd/csrc/scheduler.h, the one the server runs) and the
range pool (pool.h) with a fake executor: Poisson-like streams of jobs on 12
sequences with a byte budget, cancellations while pending and while running,
refusals (oversized job, full queue, stopped server), and a random
alloc/free stress of the pool.  It is built with g++ twice -- AddressSanitizer
+ UndefinedBehaviorSanitizer, and ThreadSanitizer -- and must exit cleanly
with no sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpu", "scheduler_fake_exec.cpp")
INC = os.path.join(ROOT, "paper_2503_22652_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_scheduler_with_fake_executor_under_sanitizer(tmp_path, san):
    exe = str(tmp_path / "sched")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fno-omit-frame-pointer",
           f"-fsanitize={san}", "-I", INC, SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout.split()
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
