"""Pins of the round-trip-time statistics oracle (Secs. IV, V) against facts outside it.

* Eq. (9) against scipy's generalized extreme value distribution (shape c = -xi), an independent
  implementation: CDF, density, quantiles, mean;
* the density as the derivative of the CDF (finite differences);
* the quantile mean of Eq. (14) (quadrature of its defining integral) against its closed form
  through the upper incomplete gamma function (mpmath), and its eps -> 0 limit against the
  distribution mean as printed in Eq. (11);
* the likelihood against scipy's log-density; the ML fit recovering the parameters of a large
  sample and sitting at a stationary point; the least-squares fit recovering the parameters
  exactly from data placed at the exact quantiles;
* the relative performance of a method whose times are c times the reference's: r = c, with no
  jackknife spread.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import stats as sst

from oracle import stats as S

CASES = [(1000.0, 300.0, 0.3), (50.0, 20.0, 0.8), (2e4, 5e3, 1.3), (10.0, 2.0, 2.5)]


def _gev(params):
    mu, beta, xi = params
    return sst.genextreme(-xi, loc=mu, scale=beta)


@pytest.mark.parametrize("params", CASES)
def test_cdf_pdf_quantile_against_scipy(params):
    g = _gev(params)
    lo = S.support_lower(*params)
    taus = lo + params[1] * np.array([1e-3, 0.1, 0.5, 1.0, 3.0, 30.0, 1e3])
    assert np.allclose(S.cdf(params, taus), g.cdf(taus), rtol=1e-9, atol=1e-300)
    assert np.allclose(S.pdf(params, taus), g.pdf(taus), rtol=1e-9, atol=1e-300)
    assert S.cdf(params, lo - 1.0) == 0.0
    for p in (1e-6, 0.01, 0.5, 0.9, 0.9999):
        q = S.quantile(params, p)
        assert q == pytest.approx(g.ppf(p), rel=1e-10)
        assert float(S.cdf(params, q)) == pytest.approx(p, rel=1e-10)


@pytest.mark.parametrize("params", CASES)
def test_pdf_is_the_derivative_of_the_cdf(params):
    lo = S.support_lower(*params)
    for t in lo + params[1] * np.array([0.2, 1.0, 5.0]):
        h = 1e-5 * params[1]
        fd = (S.cdf(params, t + h) - S.cdf(params, t - h)) / (2 * h)
        assert float(S.pdf(params, t)) == pytest.approx(float(fd), rel=1e-6)


@pytest.mark.parametrize("params", CASES)
@pytest.mark.parametrize("eps", [1e-4, 1e-2, 0.3])
def test_quantile_mean_closed_form(params, eps):
    mu, beta, xi = params
    with mpmath.workdps(30):
        closed = (mu - beta / xi) * (1 - eps) + beta / xi * mpmath.gammainc(1 - xi, -mpmath.log(1 - mpmath.mpf(eps)))
    assert S.quantile_mean(params, eps) == pytest.approx(float(closed), rel=1e-12)


@pytest.mark.parametrize("params", [c for c in CASES if c[2] < 1])
def test_mean_is_eq11_and_the_eps0_limit(params):
    mu, beta, xi = params
    eq11 = mu + beta / xi * (math.gamma(1 - xi) - 1)
    assert S.quantile_mean(params, 0.0) == pytest.approx(eq11, rel=1e-12)
    assert S.quantile_mean(params, 0.0) == pytest.approx(_gev(params).mean(), rel=1e-10)
    # the tail left out beyond Q(1 - eps) is of order beta eps^(1 - xi)
    assert abs(S.quantile_mean(params, 1e-12) - eq11) < 10 * beta * 1e-12 ** (1 - xi)


def test_quantile_mean_diverges_for_xi_at_least_one():
    params = (2e4, 5e3, 1.3)
    assert S.quantile_mean(params, 0.0) == math.inf
    a, b = S.quantile_mean(params, 1e-4), S.quantile_mean(params, 1e-6)
    # the tail integral grows like eps^(1 - xi)
    assert b / a == pytest.approx(100 ** 0.3, rel=0.05)


def test_nll_against_scipy_logpdf():
    rng = np.random.default_rng(3)
    params = (1000.0, 300.0, 0.45)
    t = _gev(params).rvs(size=400, random_state=rng)
    assert S.nll(params, t) == pytest.approx(-float(np.sum(_gev(params).logpdf(t))), rel=1e-12)
    assert S.nll((params[0] + 1e6, params[1], params[2]), t) == math.inf   # support above a sample


def test_ml_fit_recovers_and_is_stationary():
    rng = np.random.default_rng(11)
    true = (1000.0, 300.0, 0.4)
    t = _gev(true).rvs(size=20000, random_state=rng)
    (mu, beta, xi), f = S.fit_ml(t)
    assert mu == pytest.approx(true[0], rel=0.02)
    assert beta == pytest.approx(true[1], rel=0.05)
    assert xi == pytest.approx(true[2], abs=0.03)
    for k, h in ((0, 1e-3), (1, 1e-3), (2, 1e-6)):
        v = [mu, beta, xi]
        up, dn = list(v), list(v)
        up[k] += h
        dn[k] -= h
        g = (S.nll(up, t) - S.nll(dn, t)) / (2 * h)
        assert abs(g) * (abs(v[k]) + 1) < 1e-2 * len(t)


def test_ls_fit_exact_on_exact_quantiles():
    true = (500.0, 120.0, 0.7)
    n = 300
    t = _gev(true).ppf((np.arange(n) + 0.5) / n)
    (mu, beta, xi), f = S.fit_ls(t)
    assert f < 1e-20
    assert mu == pytest.approx(true[0], rel=1e-7)
    assert beta == pytest.approx(true[1], rel=1e-7)
    assert xi == pytest.approx(true[2], rel=1e-7)


def test_relative_performance_of_scaled_times():
    rng = np.random.default_rng(5)
    ref = _gev((200.0, 60.0, 0.5)).rvs(size=24, random_state=rng)
    r = S.relative_performance(3.0 * ref, ref, eps=1e-4, method=0, blocks=6)
    assert r["r_pop"] == pytest.approx(3.0, rel=1e-13)
    assert r["r_pop_err"] < 1e-12
    assert r["r_eps"] == pytest.approx(3.0, rel=1e-6)
    assert r["r_eps_err"] < 1e-5
    other = _gev((200.0, 60.0, 0.5)).rvs(size=24, random_state=rng)
    r2 = S.relative_performance(other, ref, eps=1e-4, method=0, blocks=6)
    assert r2["r_pop_err"] > 1e-3


@pytest.mark.parametrize("eps", [0.0, 1e-4, 0.3])
def test_quantile_mean_gumbel_limit(eps):
    # xi -> 0 is the Gumbel law: the quantile mean tends to the Gumbel one (scipy's quadrature
    # of x f(x) up to the Gumbel quantile, unnormalized; at eps = 0 the mean mu + beta gamma)
    mu, beta = 184.76, 35.5
    g = sst.gumbel_r(loc=mu, scale=beta)
    want = mu + beta * np.euler_gamma if eps == 0.0 else g.expect(lambda x: x, ub=g.ppf(1 - eps))
    assert S.quantile_mean((mu, beta, 1e-10), eps) == pytest.approx(want, rel=1e-8)
