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
    assert bench.ALG_OPS_PER_ATTEMPT == 45.0
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'default="c4"' in src


def test_first_convergence_summary():
    import numpy as np
    import bench
    Ls = [4] * 5 + [12] * 4
    first = np.array([1, 2, 2, 3, -1, -1, -1, 7, -1])
    s = {d["L"]: d for d in bench.first_convergence_summary(first, Ls, cap=10)}
    assert s[4] == {"L": 4, "realizations": 5, "converged": 4, "censored": 1, "median": 2, "p90": ">10"}
    assert s[12]["converged"] == 1 and s[12]["censored"] == 3 and s[12]["median"] == ">10"


def test_counter_summary_matches_workload_kernel_and_source(tmp_path, monkeypatch):
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    digest = bench.kernel_source_digest()
    (tmp_path / "profiles" / "k_x_traffic.txt").write_text(
        "# comment: not a key\nkernel: k_sweeps_queue\nconfig: c4\nsweeps_per_launch: 1024\n"
        f"traffic_bytes_per_launch: 123.5\nsource_sha256: {digest}\n")
    assert bench.counter_summary("c4", "k_sweeps_queue", 1024, "traffic_bytes_per_launch") == 123.5
    assert bench.counter_summary("c4", "k_sweeps_queue", 256, "traffic_bytes_per_launch") is None
    assert bench.counter_summary("c3", "k_sweeps_queue", 1024, "traffic_bytes_per_launch") is None
    assert bench.counter_summary("c4", "k_sweeps_queue", 1024, "valu_lane_instructions_per_attempt") is None
    assert bench.counter_summary("c4", "k_sweeps_queue", None, "traffic_bytes_per_launch") == 123.5
    (tmp_path / "profiles" / "k_x_traffic.txt").write_text(
        "kernel: k_sweeps_queue\nconfig: c4\nsweeps_per_launch: 1024\ntraffic_bytes_per_launch: 1\n"
        "source_sha256: 00\n")
    assert bench.counter_summary("c4", "k_sweeps_queue", 1024, "traffic_bytes_per_launch") is None


def test_cpu_baseline_runs_the_oracle_for_mixed_and_tempering_workloads(orc):
    import bench
    for mix, prof in ((bench.MIX_C4[:3], bench.PROFILES["c4"]), ([(4, 8)], None)):
        r = bench.cpu_baseline(mix, 64, prof, seconds_target=0.3)
        assert r["kind"] == "oracle" and r["value"] > 0 and r["cores"] >= 1
        assert r["nproc"] >= r["cores"] and r["cpu_model"]
