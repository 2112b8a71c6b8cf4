"""Oracle of the round-trip-time statistics (Secs. IV, V): test infrastructure, not product code.

Written from the definitions: the Frechet CDF of Eq. (9), its density, the distribution mean of
Eq. (10) and the quantile mean of Eq. (14) as the integrals they are defined by (mpmath
quadrature, in the variable p = F(tau)), the quantile function of Eq. (13) as the inverse of Eq. (9), maximum-likelihood and
least-squares fits as the optima of their objectives (scipy's optimizers as steps), and the
relative performance r of Table I with a delete-a-block jackknife (the paper names the jackknife
without its variant). Only the tests and the CPU leg of the benchmark use this module.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np
from scipy import optimize, stats


def support_lower(mu, beta, xi):
    return mu - beta / xi


def cdf(params, tau):
    """Eq. (9): exp(-(1 + xi (tau - mu)/beta)^(-1/xi)); 0 below the support."""
    mu, beta, xi = params
    z = 1.0 + xi * (np.asarray(tau, dtype=np.float64) - mu) / beta
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.exp(-np.power(np.where(z > 0, z, 1.0), -1.0 / xi))
    return np.where(z > 0, out, 0.0)


def pdf(params, tau):
    """dF/dtau of Eq. (9)."""
    mu, beta, xi = params
    z = 1.0 + xi * (np.asarray(tau, dtype=np.float64) - mu) / beta
    zz = np.where(z > 0, z, 1.0)
    out = (1.0 / beta) * np.power(zz, -1.0 - 1.0 / xi) * np.exp(-np.power(zz, -1.0 / xi))
    return np.where(z > 0, out, 0.0)


def quantile(params, p):
    """Eq. (13): the inverse of Eq. (9), found by bisection on the CDF (not the printed form)."""
    mu, beta, xi = params
    lo = support_lower(mu, beta, xi)
    hi = lo + beta
    while cdf(params, hi) < p:
        hi = lo + 2.0 * (hi - lo)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if cdf(params, mid) < p:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _mp_pdf(params):
    mu, beta, xi = (mpmath.mpf(v) for v in params)

    def f(t):
        z = 1 + xi * (t - mu) / beta
        if z <= 0:
            return mpmath.mpf(0)
        return (1 / beta) * z ** (-1 - 1 / xi) * mpmath.exp(-z ** (-1 / xi))
    return f


def quantile_mean(params, eps, dps=30):
    """Eq. (14): the integral of tau f(tau) from the lower end of the support to Q(1 - eps)
    (eps = 0: the distribution mean of Eq. (10), inf for xi >= 1), taken in the variable p = F(tau)
    as the integral of Q(p) over [0, 1 - eps] -- the same integral after the substitution, with Q
    the algebraic inverse of Eq. (9), mu + beta (z - 1)/xi, z = (-ln p)^(-xi) -- by quadrature
    in s = -ln(1 - p), with breakpoints every ln 10 in s. In p the integrand stays bounded in size for any xi > 0
    (in tau the density's exponent 1/xi overflows as xi -> 0, the Gumbel limit)."""
    mu, beta, xi = params
    if eps == 0.0 and xi >= 1.0:
        return math.inf
    with mpmath.workdps(dps):
        mu_m, beta_m, xi_m = (mpmath.mpf(v) for v in params)

        def integrand(s):
            # u = 1 - p = e^-s, so dp = -e^-s ds; -ln p stays accurate at both ends, and
            # (z - 1)/xi with z = exp(-xi ln(-ln p)) is formed without cancellation for small xi
            if s <= 0:
                return mpmath.mpf(0)
            ln_p = mpmath.log(-mpmath.expm1(-s)) if s < 1 else mpmath.log1p(-mpmath.exp(-s))
            Qp = mu_m + beta_m * mpmath.expm1(-xi_m * mpmath.log(-ln_p)) / xi_m
            return Qp * mpmath.exp(-s)
        # s over [0, -ln eps] (to infinity for eps = 0), with breakpoints every ln 10
        top = mpmath.inf if eps == 0.0 else -mpmath.log(mpmath.mpf(eps))
        pts = [mpmath.mpf(0), mpmath.log(2)]
        k = 1
        while k * mpmath.log(10) < top and k <= 200:
            pts.append(k * mpmath.log(10))
            k += 1
        pts.append(top)
        return float(mpmath.quad(integrand, pts))


def nll(params, tau):
    """Negative log-likelihood of the sample under Eq. (9)'s density (inf outside the support)."""
    mu, beta, xi = params
    if beta <= 0 or xi <= 0:
        return math.inf
    z = 1.0 + xi * (np.asarray(tau, dtype=np.float64) - mu) / beta
    if np.any(z <= 0):
        return math.inf
    return float(np.sum(np.log(beta) + (1.0 + 1.0 / xi) * np.log(z) + np.power(z, -1.0 / xi)))


def fit_ml(tau):
    """Maximum likelihood. The times are divided by their median first (the fit is then exactly
    scale-equivariant) and the oracle's own negative log-likelihood is minimised by Nelder-Mead
    from several starts -- scipy's GEV fit (shape c = -xi) and shapes xi = 0.2, 0.5, 1, 2 with
    location and scale matching the sample median and interquartile range -- keeping the best."""
    t0 = np.asarray(tau, dtype=np.float64)
    sc = float(np.median(t0))
    t = t0 / sc
    obj = lambda v: nll((v[0], math.exp(v[1]), math.exp(v[2])), t)
    starts = []
    c, loc, scale = stats.genextreme.fit(t)
    starts.append((loc, scale, max(-c, 1e-3)))
    q1, q2, q3 = np.quantile(t, [0.25, 0.5, 0.75])
    for xi in (0.2, 0.5, 1.0, 2.0):
        # Eq. (9) inverted at p = 1/4, 1/2, 3/4 for this xi: the spread fixes beta, the median mu
        g = lambda p: ((-math.log(p)) ** (-xi) - 1.0) / xi
        beta = (q3 - q1) / (g(0.75) - g(0.25))
        starts.append((q2 - beta * g(0.5), beta, xi))
    opts = {"xatol": 1e-12, "fatol": 1e-13, "maxiter": 40000, "maxfev": 80000}
    best = None
    for mu, beta, xi in starts:
        low = mu - beta / xi
        if low >= t.min():
            mu -= (low - t.min()) + 1e-3 * beta
        r = optimize.minimize(obj, [mu, math.log(beta), math.log(xi)], method="Nelder-Mead", options=opts)
        for _ in range(5):   # restart from the optimum until it no longer improves
            r2 = optimize.minimize(obj, r.x, method="Nelder-Mead", options=opts)
            if r2.fun >= r.fun - 1e-13 * abs(r.fun):
                break
            r = r2
        if best is None or r.fun < best.fun:
            best = r
    v = best.x
    # back to the original scale: mu and beta scale with the times, the likelihood gains n ln(sc)
    return (float(v[0] * sc), float(math.exp(v[1]) * sc), float(math.exp(v[2]))), float(best.fun + len(t) * math.log(sc))


def fit_ls(tau):
    """Least squares between Eq. (9) and the plotting positions (i - 1/2)/n of the sorted sample."""
    t = np.sort(np.asarray(tau, dtype=np.float64))
    n = len(t)
    pos = (np.arange(n) + 0.5) / n
    (mu0, beta0, xi0), _ = fit_ml(t)
    res = lambda v: cdf((v[0], math.exp(v[1]), math.exp(v[2])), t) - pos
    r = optimize.least_squares(res, [mu0, math.log(beta0), math.log(xi0)], xtol=1e-15, ftol=1e-15, gtol=1e-15,
                               max_nfev=20000)
    v = r.x
    return (float(v[0]), float(math.exp(v[1])), float(math.exp(v[2]))), float(np.sum(r.fun ** 2))


def relative_performance(tau_m, tau_ref, eps=1e-4, method=0, blocks=0):
    """r_pop = ratio of population means, r_eps = ratio of fitted quantile means (Table I), each
    with the jackknife error over `blocks` contiguous blocks of realizations left out in turn
    (0: one realization per block): err^2 = (B-1)/B sum_b (r_b - mean_b r_b)^2."""
    a = np.asarray(tau_m, dtype=np.float64)
    b = np.asarray(tau_ref, dtype=np.float64)
    n = len(a)
    B = n if blocks == 0 else blocks
    fit = fit_ml if method == 0 else fit_ls

    def est(keep):
        pa, _ = fit(a[keep])
        pb, _ = fit(b[keep])
        return a[keep].mean() / b[keep].mean(), quantile_mean(pa, eps) / quantile_mean(pb, eps), pa, pb

    rp, re, pa, pb = est(np.ones(n, bool))
    jp, je = [], []
    for k in range(B):
        keep = np.ones(n, bool)
        keep[k * n // B:(k + 1) * n // B] = False
        x, y, _, _ = est(keep)
        jp.append(x)
        je.append(y)

    def err(v):
        v = np.asarray(v)
        return math.sqrt((B - 1) / B * float(np.sum((v - v.mean()) ** 2)))
    return {"r_pop": rp, "r_pop_err": err(jp), "r_eps": re, "r_eps_err": err(je), "fit_m": pa, "fit_ref": pb,
            "blocks": B}


def running_mean(tau):
    """Eq. (12): tau_bar(n) = (1/n) sum_{i=1..n} tau_i for n = 1..N, in the order given."""
    out = []
    s = 0.0
    for i, t in enumerate(np.asarray(tau, dtype=np.float64)):
        s += float(t)
        out.append(s / (i + 1))
    return np.array(out)


def ks_distance(params, tau):
    """sup over tau of |F_n(tau) - F(tau)| between the empirical CDF F_n of the sample and Eq. (9):
    the step function F_n jumps only at the sample points, so the supremum is attained at one of
    them, from the left (F_n = count below) or from the right (F_n = count at or below)."""
    t = np.asarray(tau, dtype=np.float64)
    n = len(t)
    d = 0.0
    for x in t:
        below = float(np.sum(t < x)) / n
        at_or_below = float(np.sum(t <= x)) / n
        f = float(cdf(params, x))
        d = max(d, abs(f - below), abs(at_or_below - f))
    return d


def jackknife(stat, n, blocks=0):
    """Delete-a-block jackknife of a statistic of n ordered observations: stat(keep) is evaluated
    on the full sample and with each of B contiguous blocks [b n / B, (b + 1) n / B) left out
    (B = n for blocks = 0); err^2 = (B - 1)/B sum_b (theta_b - mean_b theta_b)^2, per component."""
    B = n if blocks == 0 else blocks
    full = np.atleast_1d(np.asarray(stat(np.ones(n, bool)), dtype=np.float64))
    parts = []
    for k in range(B):
        keep = np.ones(n, bool)
        keep[k * n // B:(k + 1) * n // B] = False
        parts.append(np.atleast_1d(np.asarray(stat(keep), dtype=np.float64)))
    parts = np.array(parts)
    err = np.sqrt((B - 1) / B * np.sum((parts - parts.mean(axis=0)) ** 2, axis=0))
    return full, err, B


def fit_jackknife(tau, method=0, blocks=0):
    """The Frechet fit of Eq. (9) to the sample and the jackknife errors of (mu, beta, xi) over
    blocks of realizations (Fig. 4: the shape xi per size and method with jackknife errors)."""
    t = np.asarray(tau, dtype=np.float64)
    fit = fit_ml if method == 0 else fit_ls
    full, err, B = jackknife(lambda keep: fit(t[keep])[0], len(t), blocks)
    return tuple(float(x) for x in full), tuple(float(x) for x in err), B
