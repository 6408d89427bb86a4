"""CPU test of the serving queue's scheduling policy (admission against a device-memory budget,
slot reuse and eviction, arrival order, failure handling, group pass alignment).

The policy is host code in ``paper_2607_06021_amd/csrc/serve_policy.h``, the same templates the
server instantiates; ``tests/sched_check.cpp`` drives them with fake slots, a fake budget and a
fake clock. It is built here with g++ under AddressSanitizer and UndefinedBehaviorSanitizer, so
a leak, an out-of-bounds access or undefined behaviour in the policy fails the test as well.
"""

import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parent.parent
SRC = ROOT / "tests" / "sched_check.cpp"
INC = ROOT / "paper_2607_06021_amd" / "csrc"


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_serving_policy_under_sanitizers(tmp_path):
    exe = tmp_path / "sched_check"
    build = subprocess.run(
        ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-I", str(INC), str(SRC), "-o", str(exe)],
        capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-4000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                         env={"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-4000:]
    assert "ALL OK" in run.stdout, out[-4000:]
    for case in ("budget_exhausted_queues", "fifo_no_overtake", "create_failure",
                 "failed_request_frees_slot", "lru_eviction", "random_stream", "plan_group",
                 "group_alignment"):
        assert f"ok {case}" in run.stdout
