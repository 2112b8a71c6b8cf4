// Round-trip-time statistics across disorder realizations (Secs. IV, V): the Frechet form of the
// distribution of the realizations' mean round-trip times, Eq. (9); its mean, Eq. (11); the
// quantile function, Eq. (13); the quantile mean, Eq. (14), in closed form; fits of the three
// parameters to measured times, with delete-a-block jackknife errors (the shape per size and
// method, Fig. 4); the distance between the empirical and the fitted distribution (Fig. 3); the
// running mean of Eq. (12) (Fig. 5); and the relative performance of two methods with
// delete-a-block jackknife errors (Sec. V, Table I). Host code only: a few thousand numbers per fit.
#include <algorithm>
#include <array>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "../../include/nfm.h"

namespace {

thread_local std::string g_err;

nfm_status fail(const std::string& m) {
  g_err = m;
  return NFM_EINVAL;
}

constexpr double kInf = std::numeric_limits<double>::infinity();
constexpr double kEulerGamma = 0.57721566490153286061;

// Upper incomplete gamma for a > 0 or a == 0 (then E1), x > 0.
double upper_gamma_base(double a, double x) {
  if (a > 0.0 && x < a + 1.0) {
    // lower part by its series: gamma(a, x) = x^a e^-x sum_n x^n / (a (a+1) ... (a+n))
    double term = 1.0 / a, sum = term;
    for (int n = 1; n < 100000; ++n) {
      term *= x / (a + n);
      sum += term;
      if (std::fabs(term) <= std::fabs(sum) * 1e-17) break;
    }
    return std::tgamma(a) - std::exp(a * std::log(x) - x) * sum;
  }
  if (a == 0.0 && x <= 1.0) {
    // E1(x) = -gamma_E - ln x - sum_k (-x)^k / (k k!)
    double term = 1.0, sum = 0.0;
    for (int k = 1; k < 1000; ++k) {
      term *= -x / k;
      const double t = term / k;
      sum += t;
      if (std::fabs(t) <= std::fabs(sum) * 1e-17) break;
    }
    return -kEulerGamma - std::log(x) - sum;
  }
  // continued fraction (modified Lentz) of Gamma(a, x) = x^a e^-x / (x + 1 - a - 1 (1 - a) / (x + 3 - a - ...))
  const double tiny = 1e-300;
  double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i < 100000; ++i) {
    const double an = -i * (i - a);
    b += 2.0;
    d = an * d + b;
    if (std::fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (std::fabs(del - 1.0) < 1e-16) break;
  }
  return std::exp(a * std::log(x) - x) * h;
}

struct Params {
  double mu, beta, xi;
};

double cdf(const Params& d, double tau) {
  const double z = 1.0 + d.xi * (tau - d.mu) / d.beta;
  if (z <= 0.0) return 0.0;
  return std::exp(-std::pow(z, -1.0 / d.xi));
}

// negative log-likelihood of the sample (+inf outside the support or for beta, xi <= 0)
double nll(const std::vector<double>& t, const Params& d) {
  if (!(d.beta > 0.0) || !(d.xi > 0.0)) return kInf;
  const double lb = std::log(d.beta), e = 1.0 + 1.0 / d.xi;
  double s = 0.0;
  for (double x : t) {
    const double z = 1.0 + d.xi * (x - d.mu) / d.beta;
    if (!(z > 0.0)) return kInf;
    const double lz = std::log(z);
    s += lb + e * lz + std::exp(-lz / d.xi);
  }
  return s;
}

// least squares between the CDF and the plotting positions (i - 1/2)/n of the sorted sample
double lsq(const std::vector<double>& sorted, const Params& d) {
  if (!(d.beta > 0.0) || !(d.xi > 0.0)) return kInf;
  const double n = (double)sorted.size();
  double s = 0.0;
  for (size_t i = 0; i < sorted.size(); ++i) {
    const double r = cdf(d, sorted[i]) - (i + 0.5) / n;
    s += r * r;
  }
  return s;
}

double quantile_of_sorted(const std::vector<double>& s, double p) {
  const double pos = p * (double)(s.size() - 1);
  const size_t i = (size_t)pos;
  if (i + 1 >= s.size()) return s.back();
  return s[i] + (pos - (double)i) * (s[i + 1] - s[i]);
}

// Starting points: the quantile function through the sample quartiles, with xi from their
// spacing ratio (bisection) and with xi = 0.2, 0.5, 1, 2 (beta/xi from the interquartile range,
// mu from the median), each moved left where needed so that the support holds every sample.
std::vector<Params> starting_points(const std::vector<double>& s) {
  const double q1 = quantile_of_sorted(s, 0.25), q2 = quantile_of_sorted(s, 0.5), q3 = quantile_of_sorted(s, 0.75);
  const double A1 = -std::log(0.25), A2 = -std::log(0.5), A3 = -std::log(0.75);
  auto ratio = [&](double xi) {
    return (std::pow(A3, -xi) - std::pow(A2, -xi)) / (std::pow(A2, -xi) - std::pow(A1, -xi));
  };
  const double R = (q3 - q2) / std::max(q2 - q1, 1e-300 + 1e-12 * std::fabs(q2));
  double lo = 1e-3, hi = 20.0, xr = 0.5;
  if (R <= ratio(lo)) xr = lo;
  else if (R >= ratio(hi)) xr = hi;
  else {
    for (int it = 0; it < 200; ++it) {
      xr = 0.5 * (lo + hi);
      (ratio(xr) < R ? lo : hi) = xr;
    }
  }
  std::vector<Params> out;
  for (double xi : {xr, 0.2, 0.5, 1.0, 2.0}) {
    double bx = (q3 - q1) / (std::pow(A3, -xi) - std::pow(A1, -xi));   // beta / xi
    if (!(bx > 0.0) || !std::isfinite(bx)) bx = std::max(q3 - q1, 1e-12 * std::fabs(q2) + 1e-300);
    Params d{q2 - bx * (std::pow(A2, -xi) - 1.0), bx * xi, xi};
    const double lower = d.mu - bx;   // support starts at mu - beta/xi
    if (!(lower < s.front())) d.mu -= (lower - s.front()) + 1e-3 * (q3 - q1 + std::fabs(s.front()) * 1e-9);
    out.push_back(d);
  }
  return out;
}

// Nelder-Mead on (mu, ln beta, ln xi), restarted from its best point until a restart no longer
// improves the objective.
template <class F>
Params minimize(F&& f, Params start, double* fbest) {
  using V = std::array<double, 3>;
  auto to_p = [](const V& v) { return Params{v[0], std::exp(v[1]), std::exp(v[2])}; };
  auto eval = [&](const V& v) {
    const double y = f(to_p(v));
    return std::isfinite(y) ? y : kInf;
  };
  V x0{start.mu, std::log(start.beta), std::log(start.xi)};
  double best = eval(x0);
  for (int restart = 0; restart < 20; ++restart) {
    std::array<V, 4> S;
    std::array<double, 4> Y;
    S[0] = x0;
    const double scale_mu = 0.1 * std::max(std::fabs(start.beta), 1e-12 * (std::fabs(x0[0]) + 1.0));
    for (int k = 0; k < 3; ++k) {
      S[k + 1] = x0;
      S[k + 1][k] += (k == 0) ? scale_mu : 0.1;
    }
    for (int k = 0; k < 4; ++k) Y[k] = eval(S[k]);
    for (int it = 0; it < 20000; ++it) {
      std::array<int, 4> o{0, 1, 2, 3};
      std::sort(o.begin(), o.end(), [&](int a, int b) { return Y[a] < Y[b]; });
      std::array<V, 4> S2;
      std::array<double, 4> Y2;
      for (int k = 0; k < 4; ++k) {
        S2[k] = S[o[k]];
        Y2[k] = Y[o[k]];
      }
      S = S2;
      Y = Y2;
      const double spread = std::fabs(Y[3] - Y[0]);
      double size = 0.0;
      for (int k = 1; k < 4; ++k)
        for (int j = 0; j < 3; ++j) {
          const double sc = (j == 0) ? std::max(std::fabs(S[0][0]), std::exp(S[0][1])) : 1.0;
          size = std::max(size, std::fabs(S[k][j] - S[0][j]) / sc);
        }
      if (spread <= 1e-14 * (std::fabs(Y[0]) + 1e-300) && size < 1e-10) break;
      V c{0, 0, 0};
      for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) c[j] += S[k][j] / 3.0;
      auto along = [&](double t) {
        V v;
        for (int j = 0; j < 3; ++j) v[j] = c[j] + t * (S[3][j] - c[j]);
        return v;
      };
      const V xr = along(-1.0);
      const double yr = eval(xr);
      if (yr < Y[0]) {
        const V xe = along(-2.0);
        const double ye = eval(xe);
        if (ye < yr) {
          S[3] = xe;
          Y[3] = ye;
        } else {
          S[3] = xr;
          Y[3] = yr;
        }
      } else if (yr < Y[2]) {
        S[3] = xr;
        Y[3] = yr;
      } else {
        const bool outside = yr < Y[3];
        const V xc = along(outside ? -0.5 : 0.5);
        const double yc = eval(xc);
        if (yc < (outside ? yr : Y[3])) {
          S[3] = xc;
          Y[3] = yc;
        } else {
          for (int k = 1; k < 4; ++k) {
            for (int j = 0; j < 3; ++j) S[k][j] = S[0][j] + 0.5 * (S[k][j] - S[0][j]);
            Y[k] = eval(S[k]);
          }
        }
      }
    }
    int ib = 0;
    for (int k = 1; k < 4; ++k)
      if (Y[k] < Y[ib]) ib = k;
    const bool improved = Y[ib] < best - 1e-13 * std::fabs(best);
    if (Y[ib] <= best) {
      best = Y[ib];
      x0 = S[ib];
    }
    if (!improved && restart > 0) break;
  }
  *fbest = best;
  return to_p(x0);
}

// The fit runs on the times divided by their median (so that it is scale-equivariant), from
// every starting point, keeping the best optimum; then back to the original scale.
Params fit(const std::vector<double>& sorted, int method, double* objective) {
  const double sc = quantile_of_sorted(sorted, 0.5);
  std::vector<double> u(sorted.size());
  for (size_t i = 0; i < u.size(); ++i) u[i] = sorted[i] / sc;
  Params best{0, 0, 0};
  double fbest = kInf;
  for (const Params& g : starting_points(u)) {
    double f = kInf;
    const Params p = method == 0 ? minimize([&](const Params& d) { return nll(u, d); }, g, &f)
                                 : minimize([&](const Params& d) { return lsq(u, d); }, g, &f);
    if (f < fbest) {
      fbest = f;
      best = p;
    }
  }
  // the negative log-likelihood of the original times gains n ln(sc); the squares do not change
  *objective = method == 0 ? fbest + (double)u.size() * std::log(sc) : fbest;
  return Params{best.mu * sc, best.beta * sc, best.xi};
}

bool valid_sample(const double* t, int64_t n) {
  if (!t || n < 3) return false;
  for (int64_t i = 0; i < n; ++i)
    if (!(t[i] > 0.0) || !std::isfinite(t[i])) return false;
  return true;
}

// Nodes and weights of the 20-point Gauss-Legendre rule on [-1, 1] (Newton on P_20 from the
// Chebyshev-like first guesses, the textbook construction).
struct GaussLegendre20 {
  double x[20], w[20];
  GaussLegendre20() {
    const int n = 20;
    for (int i = 0; i < n; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;   // P_0, P_1, then up the three-term recurrence to P_n
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

// (Gamma(1 - xi, x) - Gamma(1, x)) / xi = int_x^inf (t^-xi - 1)/xi e^-t dt, for small xi, where the
// difference of the two gamma values cancels: in v = ln t the integrand expm1(-xi v)/xi exp(v - e^v)
// is smooth and below 1e-18 outside [-45, 4]; composite 20-point Gauss-Legendre on panels of 1/2.
double gamma_order_slope(double xi, double x) {
  static const GaussLegendre20 gl;
  const double v0 = x > 0.0 ? std::max(std::log(x), -45.0) : -45.0, v1 = 4.0;
  if (v0 >= v1) return 0.0;
  const int panels = std::max(1, (int)std::ceil((v1 - v0) / 0.5));
  const double h = (v1 - v0) / panels;
  double sum = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double c = v0 + (p + 0.5) * h;
    double part = 0.0;
    for (int i = 0; i < 20; ++i) {
      const double v = c + 0.5 * h * gl.x[i];
      part += gl.w[i] * std::expm1(-xi * v) / xi * std::exp(v - std::exp(v));
    }
    sum += 0.5 * h * part;
  }
  return sum;
}

double quantile_mean(const Params& d, double eps) {
  if (eps <= 0.0 && d.xi >= 1.0) return kInf;
  const double x = eps > 0.0 ? -std::log1p(-eps) : 0.0;
  // (1 - eps) = e^-x = Gamma(1, x): mu (1 - eps) + beta/xi (Gamma(1 - xi, x) - Gamma(1, x))
  if (d.xi < 1e-2) return d.mu * (1.0 - eps) + d.beta * gamma_order_slope(d.xi, x);
  if (eps <= 0.0) return d.mu + d.beta / d.xi * (std::tgamma(1.0 - d.xi) - 1.0);
  return (d.mu - d.beta / d.xi) * (1.0 - eps) + d.beta / d.xi * nfm_upper_gamma(1.0 - d.xi, x);
}

}  // namespace

extern "C" {

const char* nfm_stats_last_error(void) { return g_err.c_str(); }

double nfm_upper_gamma(double a, double x) {
  if (!(x > 0.0) || !std::isfinite(a) || !std::isfinite(x)) return std::numeric_limits<double>::quiet_NaN();
  if (a > 0.0) return upper_gamma_base(a, x);
  // a <= 0: raise the order to a' in (0, 1] (or to 0, where Gamma(0, x) = E1(x)), then come
  // down with Gamma(s, x) = (Gamma(s + 1, x) - x^s e^-x) / s
  const double n = std::ceil(-a);
  double s = a + n;   // in [0, 1); 0 when a is a non-positive integer (start from E1)
  double g = upper_gamma_base(s, x);
  for (int k = 0; k < (int)n; ++k) {
    const double t = s - 1.0;   // go from s to s - 1
    g = (g - std::exp(t * std::log(x) - x)) / t;
    s = t;
  }
  return g;
}

double nfm_frechet_cdf(const nfm_frechet* d, double tau) {
  if (!d) return std::numeric_limits<double>::quiet_NaN();
  return cdf(Params{d->mu, d->beta, d->xi}, tau);
}

double nfm_frechet_quantile(const nfm_frechet* d, double p) {
  if (!d || !(p > 0.0) || !(p < 1.0)) return std::numeric_limits<double>::quiet_NaN();
  return d->mu + d->beta / d->xi * (std::pow(-std::log(p), -d->xi) - 1.0);
}

double nfm_frechet_mean(const nfm_frechet* d) {
  if (!d) return std::numeric_limits<double>::quiet_NaN();
  return quantile_mean(Params{d->mu, d->beta, d->xi}, 0.0);
}

double nfm_frechet_quantile_mean(const nfm_frechet* d, double eps) {
  if (!d || !(eps >= 0.0) || !(eps < 1.0)) return std::numeric_limits<double>::quiet_NaN();
  return quantile_mean(Params{d->mu, d->beta, d->xi}, eps);
}

nfm_status nfm_frechet_fit(const double* tau, int64_t n, int32_t method, nfm_frechet* out, double* objective) {
  if (!out || (method != 0 && method != 1)) return fail("frechet_fit: method must be 0 (ML) or 1 (least squares)");
  if (!valid_sample(tau, n)) return fail("frechet_fit: need n >= 3 finite positive times");
  std::vector<double> s(tau, tau + n);
  std::sort(s.begin(), s.end());
  if (s.front() == s.back()) return fail("frechet_fit: all times equal");
  double obj = 0.0;
  const Params p = fit(s, method, &obj);
  if (!std::isfinite(obj)) return fail("frechet_fit: no point of finite objective found");
  *out = nfm_frechet{p.mu, p.beta, p.xi};
  if (objective) *objective = obj;
  return NFM_OK;
}

nfm_status nfm_relative_performance(const double* tau_m, const double* tau_ref, int64_t n, double eps, int32_t method,
                                    int32_t blocks, nfm_ratio* out) {
  if (!out) return fail("relative_performance: null output");
  if (!valid_sample(tau_m, n) || !valid_sample(tau_ref, n))
    return fail("relative_performance: need n >= 3 finite positive times for both methods");
  if (!(eps > 0.0) || !(eps < 1.0)) return fail("relative_performance: eps must lie in (0, 1)");
  if (method != 0 && method != 1) return fail("relative_performance: method must be 0 (ML) or 1 (least squares)");
  const int64_t B = blocks == 0 ? n : blocks;
  if (B < 2 || B > n) return fail("relative_performance: blocks must be 0 (one per realization) or in [2, n]");
  auto estimate = [&](int64_t skip_lo, int64_t skip_hi, double* rp, double* re, Params* fm, Params* fr) {
    std::vector<double> a, b;
    a.reserve(n);
    b.reserve(n);
    double sa = 0.0, sb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      if (i >= skip_lo && i < skip_hi) continue;
      a.push_back(tau_m[i]);
      b.push_back(tau_ref[i]);
      sa += tau_m[i];
      sb += tau_ref[i];
    }
    *rp = sa / sb;
    std::sort(a.begin(), a.end());
    std::sort(b.begin(), b.end());
    double oa, ob;
    const Params pa = fit(a, method, &oa), pb = fit(b, method, &ob);
    *re = quantile_mean(pa, eps) / quantile_mean(pb, eps);
    if (fm) *fm = pa;
    if (fr) *fr = pb;
    return std::isfinite(oa) && std::isfinite(ob);
  };
  double rp, re;
  Params fm, fr;
  if (!estimate(0, 0, &rp, &re, &fm, &fr)) return fail("relative_performance: fit failed on the full sample");
  std::vector<double> jp(B), je(B);
  for (int64_t k = 0; k < B; ++k) {
    const int64_t lo = k * n / B, hi = (k + 1) * n / B;
    if (!estimate(lo, hi, &jp[k], &je[k], nullptr, nullptr)) return fail("relative_performance: fit failed on a subsample");
  }
  auto jk_err = [&](const std::vector<double>& v) {
    double m = 0.0;
    for (double x : v) m += x;
    m /= (double)B;
    double s = 0.0;
    for (double x : v) s += (x - m) * (x - m);
    return std::sqrt((double)(B - 1) / (double)B * s);
  };
  *out = nfm_ratio{rp, jk_err(jp), re, jk_err(je), nfm_frechet{fm.mu, fm.beta, fm.xi},
                   nfm_frechet{fr.mu, fr.beta, fr.xi}, (int32_t)B, 0};
  return NFM_OK;
}

nfm_status nfm_frechet_fit_jackknife(const double* tau, int64_t n, int32_t method, int32_t blocks, nfm_frechet* fit_out,
                                     nfm_frechet* err_out, int32_t* blocks_used) {
  if (!fit_out || !err_out) return fail("frechet_fit_jackknife: null output");
  if (!valid_sample(tau, n)) return fail("frechet_fit_jackknife: need n >= 3 finite positive times");
  if (method != 0 && method != 1) return fail("frechet_fit_jackknife: method must be 0 (ML) or 1 (least squares)");
  const int64_t B = blocks == 0 ? n : blocks;
  if (B < 2 || B > n) return fail("frechet_fit_jackknife: blocks must be 0 (one per realization) or in [2, n]");
  if (n - (n + B - 1) / B < 3) return fail("frechet_fit_jackknife: a subsample would hold fewer than 3 times");
  auto estimate = [&](int64_t skip_lo, int64_t skip_hi, Params* out) {
    std::vector<double> a;
    a.reserve(n);
    for (int64_t i = 0; i < n; ++i)
      if (i < skip_lo || i >= skip_hi) a.push_back(tau[i]);
    std::sort(a.begin(), a.end());
    double obj;
    *out = fit(a, method, &obj);
    return std::isfinite(obj);
  };
  Params full;
  if (!estimate(0, 0, &full)) return fail("frechet_fit_jackknife: fit failed on the full sample");
  std::vector<Params> part(B);
  for (int64_t k = 0; k < B; ++k)
    if (!estimate(k * n / B, (k + 1) * n / B, &part[k])) return fail("frechet_fit_jackknife: fit failed on a subsample");
  auto jk_err = [&](double Params::*f) {
    double m = 0.0;
    for (const auto& q : part) m += q.*f;
    m /= (double)B;
    double s = 0.0;
    for (const auto& q : part) s += (q.*f - m) * (q.*f - m);
    return std::sqrt((double)(B - 1) / (double)B * s);
  };
  *fit_out = nfm_frechet{full.mu, full.beta, full.xi};
  *err_out = nfm_frechet{jk_err(&Params::mu), jk_err(&Params::beta), jk_err(&Params::xi)};
  if (blocks_used) *blocks_used = (int32_t)B;
  return NFM_OK;
}

nfm_status nfm_running_mean(const double* tau, int64_t n, double* out) {
  if (!tau || !out || n < 1) return fail("running_mean: need n >= 1 and both arrays");
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    s += tau[i];
    out[i] = s / (double)(i + 1);
  }
  return NFM_OK;
}

nfm_status nfm_frechet_ks(const nfm_frechet* d, const double* tau, int64_t n, double* dist) {
  if (!d || !tau || !dist || n < 1) return fail("frechet_ks: need a distribution, n >= 1 times and an output");
  if (!(d->beta > 0.0) || !(d->xi > 0.0)) return fail("frechet_ks: beta > 0 and xi > 0");
  std::vector<double> s(tau, tau + n);
  for (double x : s)
    if (!std::isfinite(x)) return fail("frechet_ks: times must be finite");
  std::sort(s.begin(), s.end());
  const Params p{d->mu, d->beta, d->xi};
  double D = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double F = cdf(p, s[i]);
    // the empirical CDF is i/n just below the i-th smallest time and (i+1)/n at it
    D = std::max(D, std::max(F - (double)i / (double)n, (double)(i + 1) / (double)n - F));
  }
  *dist = D;
  return NFM_OK;
}

}  // extern "C"
