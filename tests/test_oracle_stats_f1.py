"""Pins of the oracle's Sec. IV / V extras that the campaign analysis uses: the running mean of
Eq. (12) (closed form of an arithmetic sequence), the distance between the empirical CDF and the
fitted Eq. (9) (scipy's one-sample Kolmogorov-Smirnov statistic on the same CDF), and the
delete-a-block jackknife (for the sample mean it reduces to the standard error of the mean,
s / sqrt(n) delete-one and the spread of the block means with B equal blocks)."""
import math

import numpy as np
import pytest
from scipy import stats as sst

from oracle import stats as S


def test_running_mean_of_an_arithmetic_sequence():
    n = 1000
    r = S.running_mean(np.arange(1, n + 1, dtype=np.float64))
    assert np.array_equal(r, (np.arange(1, n + 1) + 1) / 2.0)
    x = np.array([3.0, 1.0, 8.0])
    assert np.allclose(S.running_mean(x), [3.0, 2.0, 4.0], rtol=0, atol=1e-15)


@pytest.mark.parametrize("params,n,seed", [((100.0, 30.0, 0.5), 50, 1), ((10.0, 2.0, 1.4), 400, 2)])
def test_ks_distance_is_scipys_statistic(params, n, seed):
    t = sst.genextreme(-params[2], loc=params[0], scale=params[1]).rvs(n, random_state=np.random.default_rng(seed))
    want = sst.kstest(t, lambda x: S.cdf(params, x)).statistic
    assert S.ks_distance(params, t) == pytest.approx(want, rel=1e-12, abs=1e-15)
    # a sample with ties: the one-sided limits at a repeated value
    tt = np.concatenate([t[:10], t[:10]])
    want = sst.kstest(tt, lambda x: S.cdf(params, x)).statistic
    assert S.ks_distance(params, tt) == pytest.approx(want, rel=1e-12, abs=1e-15)


def test_jackknife_of_the_mean():
    rng = np.random.default_rng(3)
    x = rng.exponential(5.0, 60)
    full, err, B = S.jackknife(lambda keep: x[keep].mean(), len(x), 0)
    assert B == 60 and full[0] == pytest.approx(x.mean(), rel=1e-15)
    assert err[0] == pytest.approx(x.std(ddof=1) / math.sqrt(len(x)), rel=1e-12)
    # 6 equal blocks: the standard error of the 6 block means
    full, err, B = S.jackknife(lambda keep: x[keep].mean(), len(x), 6)
    bm = x.reshape(6, 10).mean(axis=1)
    assert err[0] == pytest.approx(bm.std(ddof=1) / math.sqrt(6), rel=1e-12)


def test_fit_jackknife_spreads_with_the_sample_and_vanishes_for_identical_blocks():
    rng = np.random.default_rng(9)
    t = sst.genextreme(-0.6, loc=300.0, scale=90.0).rvs(40, random_state=rng)
    fit, err, B = S.fit_jackknife(t, 0, 8)
    assert B == 8 and all(e > 0 for e in err)
    assert fit == pytest.approx(S.fit_ml(t)[0], rel=1e-12)
    # every block the same multiset: every delete-a-block fit is the same fit
    rep = np.tile(np.sort(t[:5]), 8)
    fit, err, B = S.fit_jackknife(rep, 0, 8)
    assert max(err) < 1e-6 * max(abs(v) for v in fit)
