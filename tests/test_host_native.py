"""Host code under sanitizers (CPU only): the serving scheduler with a mock executor and a
virtual clock (admission by footprint, budget waits, continuous batching, FIFO, result
validity, forced failures, shutdown), and the planning code (validation, batches, relevance
against brute force, groups, splines).  Each program is built with g++ twice, with
AddressSanitizer + UndefinedBehaviorSanitizer and with ThreadSanitizer (the scheduler's
builder thread, the planner's threaded relevance pass), and must run clean."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_1912_06636_amd", "csrc")
INC = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
SAN = {
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"],
    "tsan": ["-fsanitize=thread"],
}
PROGRAMS = {
    "scheduler": (["scheduler_mock.cpp"], ["scheduler.cpp"], "scheduler mock: all ok"),
    "plan": (["plan_check.cpp"], ["plan.cpp"], "plan check: all ok"),
}


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("san", sorted(SAN))
@pytest.mark.parametrize("prog", sorted(PROGRAMS))
def test_host_code_under_sanitizer(tmp_path, prog, san):
    tests, srcs, done = PROGRAMS[prog]
    exe = str(tmp_path / (prog + "_" + san))
    cmd = (["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off"] + SAN[san] + INC
           + [os.path.join(NATIVE, t) for t in tests] + [os.path.join(CSRC, s) for s in srcs]
           + ["-o", exe, "-lpthread"])
    subprocess.run(cmd, check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    if san == "tsan" and "unexpected memory mapping" in r.stderr:
        pytest.skip("ThreadSanitizer runtime does not support this kernel's memory layout")
    assert r.returncode == 0, r.stdout + r.stderr
    assert done in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
