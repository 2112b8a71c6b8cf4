"""The host-side pooling of saved round-trip times (campaign --analyse): methods from several
files of the same realizations, censored entries (NaN) leaving every method's sample, and the
relative performance against the power law as the oracle computes it on the paired sample, the
jackknife errors of the fitted shape, the distance of the empirical CDF from the fit and the
running mean of Eq. (12); files of several sizes give one analysis per size."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
from scipy import stats as sst

from oracle import stats as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_analyse_pools_saved_methods(tmp_path):
    rng = np.random.default_rng(4)
    n = 48
    pl = sst.genextreme(-0.5, loc=100.0, scale=30.0).rvs(n, random_state=rng)
    flat = sst.genextreme(-0.7, loc=200.0, scale=70.0).rvs(n, random_state=rng)
    invk = sst.genextreme(-0.6, loc=150.0, scale=50.0).rvs(n, random_state=rng)
    flat[5] = np.nan      # censored under one method: dropped from every method's sample
    invk[17] = np.nan
    a, b = tmp_path / "a.npz", tmp_path / "b.npz"
    np.savez(a, tau_pl=pl, tau_flat=flat, sweeps_pl=np.int64(1000), sweeps_flat=np.int64(5000))
    np.savez(b, tau_invk=invk, sweeps_invk=np.int64(3000))
    out = subprocess.run([sys.executable, "-m", "paper_2011_08560_amd.campaign", "--analyse", str(a), str(b),
                          "--blocks", "8"], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    rec = json.loads(out.stdout)
    assert rec["censored"] == {"pl": 0, "flat": 1, "invk": 1}
    assert rec["sweeps_run"] == {"pl": 1000, "flat": 5000, "invk": 3000}
    ok = np.isfinite(flat) & np.isfinite(invk)
    assert rec["analysis"]["paired_realizations"] == int(ok.sum()) == n - 2
    for m, t in (("flat", flat), ("invk", invk)):
        want = S.relative_performance(t[ok], pl[ok], eps=1e-4, method=0, blocks=8)
        got = rec["analysis"]["methods"][m]["r"]
        assert got["r_pop"] == pytest.approx(want["r_pop"], rel=1e-12)
        assert got["r_pop_err"] == pytest.approx(want["r_pop_err"], rel=1e-9)
        assert got["r_eps"] == pytest.approx(want["r_eps"], rel=1e-4)
    assert rec["analysis"]["methods"]["pl"]["tau_pop"] == pytest.approx(float(pl[ok].mean()), rel=1e-12)
    a_pl = rec["analysis"]["methods"]["pl"]
    fit, err, B = S.fit_jackknife(pl[ok], 0, 8)
    assert a_pl["frechet_err"]["blocks"] == 8
    assert a_pl["frechet"]["xi"] == pytest.approx(fit[2], rel=1e-4)
    assert a_pl["frechet_err"]["xi"] == pytest.approx(err[2], rel=5e-3)
    assert a_pl["ks_distance"] == pytest.approx(S.ks_distance(tuple(a_pl["frechet"][k] for k in ("mu", "beta", "xi")),
                                                              pl[ok]), rel=1e-12)
    run = S.running_mean(pl[ok])
    assert np.allclose(a_pl["running_mean_series"], run, rtol=1e-14, atol=0)
    assert a_pl["running_mean"]["1"] == pytest.approx(float(pl[ok].mean()), rel=1e-12)


def test_analyse_groups_files_by_size(tmp_path):
    rng = np.random.default_rng(6)
    files = []
    for L, xi in ((4, 0.4), (6, 0.9)):
        pl = sst.genextreme(-xi, loc=100.0 * L, scale=30.0 * L).rvs(24, random_state=rng)
        flat = 2.0 * pl
        f = tmp_path / f"L{L}.npz"
        np.savez(f, tau_pl=pl, tau_flat=flat, sweeps_pl=np.int64(10), sweeps_flat=np.int64(20), L=np.int64(L))
        files.append(str(f))
    out = subprocess.run([sys.executable, "-m", "paper_2011_08560_amd.campaign", "--analyse", *files, "--blocks", "4"],
                         capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    rec = json.loads(out.stdout)
    assert sorted(rec["by_L"]) == ["4", "6"]
    for L in ("4", "6"):
        r = rec["by_L"][L]["analysis"]["methods"]["flat"]["r"]
        assert r["r_pop"] == pytest.approx(2.0, rel=1e-12)
    assert "xi = " in out.stderr and "L=6" in out.stderr


def test_scan_ratios_against_the_flat_point():
    """The exponent scan's ratios: reference = the first grid point with alpha = 0 (not the first
    point), each other point paired with it over the realizations uncensored at both, the ratios
    as the oracle computes them on that paired sample."""
    from paper_2011_08560_amd import campaign
    rng = np.random.default_rng(9)
    n = 40
    flat = sst.genextreme(-0.7, loc=200.0, scale=70.0).rvs(n, random_state=rng)
    half = sst.genextreme(-0.5, loc=90.0, scale=30.0).rvs(n, random_state=rng)
    steep = sst.genextreme(-0.9, loc=900.0, scale=300.0).rvs(n, random_state=rng)
    flat[3] = np.nan
    steep[[7, 8]] = np.nan
    grid = [{"dE": 1.0, "alpha": -0.5}, {"dE": 1.0, "alpha": 0.0}, {"dE": 1.0, "alpha": -2.0}]
    ref = campaign.scan_ratios(grid, [half, flat, steep], eps=1e-4, blocks=4)
    assert ref == 1
    assert "r_vs_reference" not in grid[1]
    for i, t in ((0, half), (2, steep)):
        ok = np.isfinite(t) & np.isfinite(flat)
        assert grid[i]["paired"] == int(ok.sum())
        want = S.relative_performance(t[ok], flat[ok], eps=1e-4, method=0, blocks=4)
        got = grid[i]["r_vs_reference"]
        assert got["r_pop"] == pytest.approx(want["r_pop"], rel=1e-12)
        assert got["r_pop_err"] == pytest.approx(want["r_pop_err"], rel=1e-9)
        assert got["r_eps"] == pytest.approx(want["r_eps"], rel=1e-4)
    assert grid[0]["paired"] == n - 1 and grid[2]["paired"] == n - 3
