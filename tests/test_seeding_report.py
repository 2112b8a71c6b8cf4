"""The paired report of the learned-start comparison on the CPU (synthetic arm records): rounds
and total sweeps to the first converged round, censoring, the same lowest level and the largest
difference of the two estimates where both converged; and the report stage over split files."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _arm(rounds, k_lo, y, k_seed):
    n = len(rounds)
    return {"rounds": np.asarray(rounds), "k_lo": np.asarray(k_lo), "k_seed": np.asarray(k_seed),
            "y": np.asarray(y, np.float32), "mask": np.ones((n, 256), np.float32)}


def test_paired_report():
    from paper_2011_08560_amd import seeding
    y0 = np.zeros((4, 256))
    plain = _arm([10, 20, 61, 30], [5, 5, 6, 7], y0, [-1] * 4)
    y1 = y0.copy()
    y1[1, 7] = 2e-3                                   # one realization differs by 2e-3 N in S/N
    seeded = _arm([2, 3, 4, 61], [5, 4, 6, 7], y1, [0, 0, -1, 0])
    r = seeding.paired_report(plain, seeded, 4, 1000, 60)
    assert r["plain"]["converged"] == 3 and r["plain"]["censored"] == 1
    assert r["seeded"]["converged"] == 3 and r["seeded"]["censored"] == 1
    assert r["both_converged"] == 2 and r["same_lowest_level"] == 1 and r["seeded_lower_level"] == 1
    assert r["seed_rejected"] == 1 and r["fewer_rounds"] == 3 and r["more_rounds"] == 1
    assert r["max_abs_dS_median"] == pytest.approx((0.0 + 2e-3 * 64) / 2, rel=1e-5)
    # sweeps: rounds x 1.1 x 1000, plus the canonical run for the seeded arm
    assert r["plain"]["sweeps_median"] == pytest.approx(np.median([11000, 22000, 67100, 33000]))
    assert r["seeded"]["sweeps_median"] == pytest.approx(np.median([2200, 3300, 4400, 67100]) + seeding.CANON_SWEEPS)


def test_report_stage_pairs_split_files(tmp_path):
    rng = np.random.default_rng(1)
    files = []
    for arm in ("plain", "seeded"):
        for first in (1_000_100, 1_000_000):           # out of order on purpose
            n = 3
            rounds = rng.integers(1, 9, n) if arm == "seeded" else rng.integers(10, 30, n)
            f = tmp_path / f"{arm}_{first}.npz"
            np.savez(f, arm=arm, first_id=np.int64(first), rounds=rounds, k_lo=np.full(n, 3),
                     k_seed=np.full(n, 0 if arm == "seeded" else -1), y=np.zeros((n, 256), np.float32),
                     mask=np.ones((n, 256), np.float32))
            files.append(str(f))
    out = subprocess.run([sys.executable, "-m", "paper_2011_08560_amd.seeding", "--stage", "report", "--eval-L", "4",
                          "--sweeps", "100", "--n-max", "40", "--inputs", *files],
                         capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    rep = json.loads(out.stdout)
    assert rep["realizations"] == 6 and rep["fewer_rounds"] == 6 and rep["same_lowest_level"] == 6
