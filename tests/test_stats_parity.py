"""Parity of the library's round-trip statistics (host code in libnfm, Secs. IV, V) with the oracle.

These functions run on the host, so they are checked on the CPU: the closed forms against the
oracle's quadratures, the incomplete gamma function against mpmath, the fits against the
oracle's fits (the library must reach an optimum at least as good, at the same parameters to
the optimizers' tolerance), and the relative performance with its jackknife errors.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import stats as sst

from oracle import stats as S

CASES = [(1000.0, 300.0, 0.3), (50.0, 20.0, 0.8), (10.0, 3.0, 1.0), (2e4, 5e3, 1.3), (10.0, 2.0, 2.5)]


@pytest.fixture(scope="module")
def nfm():
    from paper_2011_08560_amd import nfm as m
    m.lib()
    return m


def _times(params, n, seed):
    mu, beta, xi = params
    return sst.genextreme(-xi, loc=mu, scale=beta).rvs(size=n, random_state=np.random.default_rng(seed))


@pytest.mark.parametrize("params", CASES)
def test_closed_forms(nfm, params):
    mu, beta, xi = params
    lo = mu - beta / xi
    for t in lo + beta * np.array([1e-3, 0.3, 1.0, 7.0, 1e4]):
        assert nfm.frechet_cdf(params, t) == pytest.approx(float(S.cdf(params, t)), rel=1e-12, abs=1e-300)
    assert nfm.frechet_cdf(params, lo - 1.0) == 0.0
    for p in (1e-8, 0.05, 0.5, 0.99, 1 - 1e-9):
        # the oracle inverts the CDF by bisection: near p = 1 the CDF resolves tau to ~1e-16/(1 - p)
        assert nfm.frechet_quantile(params, p) == pytest.approx(S.quantile(params, p), rel=1e-9 if p < 0.999 else 1e-7)
    assert math.isnan(nfm.frechet_quantile(params, 0.0)) and math.isnan(nfm.frechet_quantile(params, 1.0))
    for eps in (1e-6, 1e-4, 1e-2, 0.3):
        assert nfm.frechet_quantile_mean(params, eps) == pytest.approx(S.quantile_mean(params, eps), rel=1e-10)
    m = nfm.frechet_mean(params)
    if xi < 1:
        assert m == pytest.approx(S.quantile_mean(params, 0.0), rel=1e-10)
    else:
        assert m == math.inf


@pytest.mark.parametrize("a", [-3.0, -2.7, -1.0, -0.5, -1e-3, 0.0, 1e-3, 0.3, 1.0, 2.5, 7.0])
@pytest.mark.parametrize("x", [1e-5, 1e-2, 0.5, 1.0, 3.0, 25.0])
def test_upper_gamma(nfm, a, x):
    with mpmath.workdps(40):
        want = float(mpmath.gammainc(a, x))
    assert nfm.upper_gamma(a, x) == pytest.approx(want, rel=1e-11)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("params,n,seed", [((1000.0, 300.0, 0.3), 60, 1), ((50.0, 20.0, 0.9), 500, 2),
                                           ((2e4, 5e3, 1.5), 2000, 3)])
def test_fit_matches_oracle(nfm, method, params, n, seed):
    t = _times(params, n, seed)
    got, f_got = nfm.frechet_fit(t, method)
    want, f_want = (S.fit_ml if method == 0 else S.fit_ls)(t)
    obj = (lambda p: S.nll(p, t)) if method == 0 else \
        (lambda p: float(np.sum((S.cdf(p, np.sort(t)) - (np.arange(n) + 0.5) / n) ** 2)))
    # the library's optimum, evaluated by the oracle, is at least as good as the oracle's
    assert obj(got) <= f_want + 1e-9 * abs(f_want) + 1e-15
    assert f_got == pytest.approx(obj(got), rel=1e-10, abs=1e-14)
    for g, w in zip(got, want):
        assert g == pytest.approx(w, rel=2e-5)


@pytest.mark.parametrize("blocks", [0, 5])
def test_relative_performance_matches_oracle(nfm, blocks):
    n = 15 if blocks == 0 else 40
    ref = _times((300.0, 90.0, 0.6), n, 7)
    m = _times((500.0, 200.0, 0.8), n, 8)
    got = nfm.relative_performance(m, ref, eps=1e-4, method=0, blocks=blocks)
    want = S.relative_performance(m, ref, eps=1e-4, method=0, blocks=blocks)
    assert got["blocks"] == want["blocks"] == (n if blocks == 0 else blocks)
    assert got["r_pop"] == pytest.approx(want["r_pop"], rel=1e-13)
    assert got["r_pop_err"] == pytest.approx(want["r_pop_err"], rel=1e-9)
    assert got["r_eps"] == pytest.approx(want["r_eps"], rel=1e-5)
    assert got["r_eps_err"] == pytest.approx(want["r_eps_err"], rel=1e-3, abs=1e-6)


def test_bad_input(nfm):
    with pytest.raises(nfm.NfmError):
        nfm.frechet_fit([1.0, 2.0], 0)
    with pytest.raises(nfm.NfmError):
        nfm.frechet_fit([1.0, -2.0, 3.0, 4.0], 0)
    with pytest.raises(nfm.NfmError):
        nfm.frechet_fit([1.0, 2.0, 3.0, np.inf], 0)
    with pytest.raises(nfm.NfmError):
        nfm.frechet_fit([1.0, 2.0, 3.0], 2)
    t = _times((300.0, 90.0, 0.6), 10, 1)
    with pytest.raises(nfm.NfmError):
        nfm.relative_performance(t, t, eps=0.0)
    with pytest.raises(nfm.NfmError):
        nfm.relative_performance(t, t, eps=1e-4, blocks=1)
    with pytest.raises(nfm.NfmError):
        nfm.relative_performance(t, t, eps=1e-4, blocks=11)
    assert math.isnan(nfm.upper_gamma(1.0, 0.0)) and math.isnan(nfm.frechet_quantile_mean((1, 1, 0.5), 1.0))


@pytest.mark.parametrize("xi", [9e-3, 1e-4, 1e-7, 1e-10])
def test_quantile_mean_near_the_gumbel_limit(nfm, xi):
    # fits of narrow round-trip-time distributions end near xi = 0, where beta/xi (Gamma(1 - xi, x)
    # - (1 - eps)) cancels; the library then integrates the difference quotient directly
    params = (184.76, 35.5, xi)
    for eps in (0.0, 1e-4, 0.3, 0.9):
        assert nfm.frechet_quantile_mean(params, eps) == pytest.approx(S.quantile_mean(params, eps), rel=1e-13)


@pytest.mark.parametrize("blocks", [0, 6])
def test_fit_jackknife_matches_oracle(nfm, blocks):
    n = 18 if blocks == 0 else 42
    t = _times((400.0, 120.0, 0.7), n, 11)
    fit, err, B = nfm.frechet_fit_jackknife(t, 0, blocks)
    wfit, werr, wB = S.fit_jackknife(t, 0, blocks)
    assert B == wB == (n if blocks == 0 else blocks)
    for g, w in zip(fit, wfit):
        assert g == pytest.approx(w, rel=2e-5)
    for g, w in zip(err, werr):
        assert g == pytest.approx(w, rel=2e-3, abs=1e-6 * max(abs(v) for v in wfit))
    with pytest.raises(nfm.NfmError):
        nfm.frechet_fit_jackknife(t[:4], 0, 2)        # a subsample of 2 times cannot be fitted


def test_running_mean_and_ks_match_oracle(nfm):
    t = _times((50.0, 20.0, 1.2), 300, 12)
    assert np.allclose(nfm.running_mean(t), S.running_mean(t), rtol=1e-14, atol=0)
    for params in ((50.0, 20.0, 1.2), (45.0, 25.0, 0.9)):
        assert nfm.frechet_ks(params, t) == pytest.approx(S.ks_distance(params, t), rel=1e-12, abs=1e-15)
    tt = np.concatenate([t[:7], t[:7], t[3:9]])      # ties
    assert nfm.frechet_ks((50.0, 20.0, 1.2), tt) == pytest.approx(S.ks_distance((50.0, 20.0, 1.2), tt), rel=1e-12)
    with pytest.raises(nfm.NfmError):
        nfm.frechet_ks((50.0, -1.0, 1.2), t)
