"""The host-side pooling of saved round-trip times (campaign --analyse): methods from several
files of the same realizations, censored entries (NaN) leaving every method's sample, and the
relative performance against the power law as the oracle computes it on the paired sample."""
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
