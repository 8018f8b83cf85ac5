"""The benchmark's contract checks that need no GPU.

One GPU is measured: more than one (by flag or by a launcher's WORLD_SIZE)
is refused with a message before anything touches a device. The HBM traffic
the benchmark reports for its dominant kernel comes from counters taken on
the kernel's current sources, so the committed figures must still match
them (a change to the kernel without new counters would report null).
"""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", BENCH)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, BENCH, *args], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_a_launcher_world_size_above_one_is_refused():
    r = _run([], {"WORLD_SIZE": "4", "RANK": "0"})
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_traffic_counters_match_the_current_kernel_sources():
    b = _bench_module()
    for kernel, e in b.TRAFFIC.items():
        assert e["digest"] == b.kernel_digest(kernel), (
            f"{kernel}: sources changed since the FETCH_SIZE / WRITE_SIZE counters were taken")
        traffic = b.measured_traffic(kernel, e["workload"], e["tuning"])
        assert traffic is not None and traffic > 0
    # a different workload or tuning never borrows the counters
    e = b.TRAFFIC["bin_kernel"]
    assert b.measured_traffic("bin_kernel", "another-workload", e["tuning"]) is None
    assert b.measured_traffic("bin_kernel", e["workload"], [2, 64, 8, 1, 1024, 0, 2]) is None
    assert b.measured_traffic("bin_kernel", e["workload"], e["tuning"][:6] + [1]) is None


def test_cobound_probe_rejects_arguments_before_any_device_call():
    """The co-bound microbenchmark checks its arguments first: out-of-range
    sizes or launch counts end with status 2 and its usage line, with no
    device touched (this container has none)."""
    import pytest
    exe = os.path.join(ROOT, "paper_2504_20937_amd", "mm_cobound")
    if not os.path.exists(exe):
        pytest.skip("mm_cobound is not built")
    for args in (["12"], ["31"], ["24", "0"], ["24", "10001"]):
        r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=60)
        assert r.returncode == 2, (args, r.returncode, r.stderr)
        assert "usage: mm_cobound" in r.stderr, r.stderr
