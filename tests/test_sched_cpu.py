"""The served form's scheduling policy on the host, under AddressSanitizer
and UndefinedBehaviorSanitizer.

``csrc/mm_sched.h`` holds the policy (per-cloud order, admission by
frame-buffer bytes, eviction, continuous batching over slots, failure
handling) with no device code. ``tests/sched/sched_check.cpp`` drives it
with a fake backend: the admission order that once left the served loop
with nothing to run (two sessions on one cloud, one buffer, submissions
A0, B0, A1), a launch that does not go out, a launch that fails on the
device, a buffer that cannot be allocated, requests arriving while a launch
is in flight, and 300 seeds of random traffic checked for order, budget,
progress and completion."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "sched", "sched_check.cpp")


def test_scheduler_policy_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "sched_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2504_20937_amd", "csrc"), SRC, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("all ok"), r.stdout
    assert "ok one_buffer_two_sessions" in r.stdout
