"""bench.py's command line on the CPU: it runs on one GPU only and says so for more, before it
touches a device; its workload table names the sizes the parity tests use."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=60, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_workloads():
    import bench
    assert bench.CONFIGS["c2"][:3] == ([(6, 1024)], 64, 100_000)
    assert bench.CONFIGS["c3"][0] == [(8, 4096)] and bench.CONFIGS["c3pt"][0] == [(8, 4096)]
    assert bench.CONFIGS["c4"][0] == [(4, 4096), (6, 2048), (8, 1024), (10, 512), (12, 256)]
    assert bench.PROFILES["c3"] == (1, 96.0, -3.6) and bench.PROFILES["c3pt"] is None
    assert bench.PEAK_LANE_OPS == 256 * 4 * 32 * 2.4e9
