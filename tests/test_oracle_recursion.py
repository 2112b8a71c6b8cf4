"""Pins for the oracle's weight recursion and ensembles (Sec. II, Eqs. (3)-(7)).

Independent facts used:
  * with the exact density of states g (enumerated at L = 3) the ensembles are
    known in closed form: W = P_SH/g yields a histogram proportional to P_SH
    (Sec. II, Eq. (4), Fig. 1), W = 1/g a flat one, and W = 1/sum_{E' <= E} g(E')
    the 1/k-ensemble (Eq. (7));
  * fed the exact steps b = ln g(k+1) - ln g(k), the oracle's weight builder must
    return S = ln g - ln g(top), the power law of Eq. (5) anchored at the ground
    state (ln P = 0 at E = 0) and the 1/k weights -ln sum_{j <= k} g(j) + const,
    each written out here from integer counts, and production under those weights
    must give the histogram each ensemble prescribes;
  * the recursion's converged estimate S(E) - S(top) must reproduce
    ln g(E) - ln g(top) within statistical error, whatever target profile
    steered the iteration;
  * the first update of a level pair reduces to the simple recursion
    lnW <- lnW - ln(H/P) (closed form on a synthetic histogram).
"""
import math

import numpy as np
import pytest

L3_REAL = 0


@pytest.fixture(scope="module")
def exact_L3(orc):
    L = 3
    J = orc.couplings(L, 20110856, L3_REAL)
    g = orc.brute_dos(L, J).astype(np.float64)
    return L, J, g


def _lnw_from_g(g, eb, k_lo, k_top, lnP):
    """lnW = -ln g + ln P on [k_lo, k_top]; levels with g = 0 (no states) take
    interpolated values, which never enter a move that can happen."""
    ks = np.arange(k_lo, k_top + 1)
    lnw = np.full(len(ks), np.nan)
    m = g[ks] > 0
    lnw[m] = -np.log(g[ks][m]) + lnP[m]
    lnw[~m] = np.interp(ks[~m], ks[m], lnw[m])
    return lnw


def _production_hist(orc, L, J, lnw, k_lo, k_top, walkers=48, burn=200, sweeps=2500):
    K, eb = orc.n_levels(L, J), orc.e_base(L, J)
    thr, row0 = orc.build_thresholds(K, lnw, k_lo, k_top)
    H = np.zeros(K, np.uint64)
    for wk in range(walkers):
        S = orc.spins(L, 21, L3_REAL, wk)
        w = orc.new_walkers(1, orc.energy(L, J, S))
        orc.muca_sweeps(L, J, S, w, thr, row0, eb + 4 * k_lo, 0, 21, L3_REAL, wk, 0, burn)
        orc.muca_sweeps(L, J, S, w, thr, row0, eb + 4 * k_lo, 0, 21, L3_REAL, wk, burn, sweeps, hist=H)
    return H.astype(np.float64)


def _levels(orc, L, J, g):
    eb = orc.e_base(L, J)
    k_lo = int(np.nonzero(g)[0][0])
    k_top = int(math.ceil(-eb / 4))
    return eb, k_lo, k_top


@pytest.mark.parametrize("kind", ["flat", "power", "invk"])
def test_exact_weights_give_target_histogram(orc, exact_L3, kind):
    L, J, g = exact_L3
    eb, k_lo, k_top = _levels(orc, L, J, g)
    ks = np.arange(k_lo, k_top + 1)
    E = (eb + 4 * ks).astype(np.float64)
    E_g = float(eb + 4 * k_lo)
    if kind == "flat":
        lnP = np.zeros(len(ks))
    elif kind == "power":
        lnP = np.array([math.log(orc.power_profile(e, E_g, 6.0, -2.0)) for e in E])
    else:
        # 1/k: W = 1/sum_{j<=k} g(j), i.e. P = g/kcum
        kcum = np.cumsum(g[ks])
        lnP = np.where(g[ks] > 0, np.log(np.maximum(g[ks], 1)) - np.log(kcum), 0.0)
    lnw = _lnw_from_g(g, eb, k_lo, k_top, lnP)
    H = _production_hist(orc, L, J, lnw, k_lo, k_top)
    m = g[ks] > 0
    h = H[ks][m] / H[ks][m].sum()
    p = np.exp(lnP[m]) / np.exp(lnP[m]).sum()
    assert np.max(np.abs(h / p - 1)) < 0.12, (kind, h / p)
    # above the top the weight is constant, so the histogram follows g there
    up = np.arange(k_top, len(g))
    up = up[g[up] > 0]
    ratio = (H[up] / H[k_top]) / (g[up] / g[k_top])
    assert np.all(np.abs(ratio[: 3] - 1) < 0.25)


def test_first_update_is_simple_recursion(orc):
    K, k_lo, k_top = 12, 2, 9
    lnW = np.zeros(K)
    lnP = np.zeros(K)
    rng = np.random.default_rng(2)
    lnW[k_lo:k_top + 1] = rng.normal(0, 1, k_top - k_lo + 1)
    H = np.zeros(K, np.uint64)
    H[k_lo:k_top + 1] = rng.integers(50, 500, k_top - k_lo + 1)
    b = np.zeros(K); p = np.zeros(K); vis = np.zeros(K, np.uint8)
    # b must equal the S steps of lnW - ln(H/P) negated: S_new = -lnW + ln H - ln P
    S_prev = np.zeros(K)
    S_prev[k_top] = 0
    for k in range(k_top - 1, k_lo - 1, -1):
        S_prev[k] = S_prev[k + 1] - b[k]
    k_new, flat = orc.rec_update(K, k_lo, k_top, k_lo, lnW, lnP, H, b, p, vis)
    assert k_new == k_lo
    Hs = H.astype(np.float64)
    for k in range(k_lo, k_top):
        simple = (math.log(Hs[k + 1]) - lnW[k + 1]) - (math.log(Hs[k]) - lnW[k])
        assert abs(b[k] - simple) < 1e-12
        assert abs(p[k] - Hs[k] * Hs[k + 1] / (Hs[k] + Hs[k + 1])) < 1e-9
    hv = Hs[k_lo:k_top + 1]
    assert abs(flat - hv.min() / hv.mean()) < 1e-12
    assert np.all(vis[k_lo:k_top + 1] == 1)


@pytest.mark.parametrize("profile,dE,alpha", [(0, 1.0, 0.0), (1, 6.0, -2.0), (2, 1.0, 0.0)])
def test_recursion_converges_to_exact_dos(orc, exact_L3, profile, dE, alpha):
    L, J, g = exact_L3
    eb, k_gs, k_top = _levels(orc, L, J, g)
    rz = orc.make_realization(L, 20110856, L3_REAL, 99, 16)
    st = orc.recursion_init(rz)
    # iterate past the first flat histogram so the accumulated estimate averages
    # down to its statistical error
    log = orc.weight_iterations(rz, st, n_iter=40, n_sweeps=1500, profile=profile, pl_dE=dE,
                                pl_alpha=alpha, f_tol=0.6, stop=False)
    assert any(r[3] for r in log), log[-6:]
    assert log[-1][2] > 0.6, log[-6:]
    assert st.k_lo == k_gs                      # the ground state was found
    S, _, _ = orc.rec_weights(rz.K, rz.eb, st.k_lo, st.k_top, profile, dE, alpha, st.b)
    ks = np.arange(st.k_lo, st.k_top + 1)
    m = g[ks] > 0
    ref = np.log(g[ks][m]) - math.log(g[k_top])
    got = S[ks][m]
    assert np.max(np.abs(got - ref)) < 0.25, np.c_[ks[m], got, ref]


def _exact_steps(g, k_lo, k_top):
    """b(k) = ln g(k+1) - ln g(k) on [k_lo, k_top), from integer counts (no gaps)."""
    K = len(g)
    b = np.zeros(K)
    assert np.all(g[k_lo:k_top + 1] > 0)
    for k in range(k_lo, k_top):
        b[k] = math.log(int(g[k + 1])) - math.log(int(g[k]))
    return b


@pytest.fixture(scope="module", params=[(3, 0), (3, 3), (2, 1), (2, 4)])
def exact_case(orc, request):
    """(L, real id): L = 3 realizations with even and odd e_base parity, and L = 2 ones whose
    level set holds E = 0 (even n_minus) or does not."""
    L, rid = request.param
    J = orc.couplings(L, 20110856, rid)
    g = orc.brute_dos(L, J)
    eb = orc.e_base(L, J)
    k_lo = int(np.nonzero(g)[0][0])
    k_top = (-eb + 3) // 4
    return L, J, g, eb, k_lo, k_top


@pytest.mark.parametrize("dE,alpha", [(6.0, -2.0), (96.0, -3.6), (1.0, -1.0), (1.0, -0.5)])
def test_rec_weights_power_law_is_eq5(orc, exact_case, dE, alpha):
    """The power-law profile of the oracle's weight builder against Eq. (5) written out:
    P_SH(E) = ((E - E_g + dE)/(dE - E_g))^alpha with E_g the lowest level of the estimate
    (the ground state here) and P_SH(0) = 1; S from the exact steps."""
    L, J, g, eb, k_lo, k_top = exact_case
    K = len(g)
    b = _exact_steps(g, k_lo, k_top)
    S, lnP, lnW = orc.rec_weights(K, eb, k_lo, k_top, 1, dE, alpha, b)
    ks = np.arange(k_lo, k_top + 1)
    E = eb + 4 * ks
    E_g = int(eb + 4 * k_lo)
    assert E_g == int(eb + 4 * np.nonzero(g)[0][0])          # anchored at the true ground state
    ref_lnP = np.array([alpha * math.log((int(e) - E_g + dE) / (dE - E_g)) for e in E])
    ref_S = np.array([math.log(int(g[k])) - math.log(int(g[k_top])) for k in ks])
    assert np.max(np.abs(S[ks] - ref_S)) <= 1e-12 * max(1.0, np.abs(ref_S).max())
    assert np.max(np.abs(lnP[ks] - ref_lnP)) <= 1e-12 * max(1.0, np.abs(ref_lnP).max())
    assert np.max(np.abs(lnW[ks] - (-ref_S + ref_lnP))) <= 1e-12 * max(1.0, np.abs(ref_S).max())
    # P decreases from the ground state upwards (alpha < 0) and is 1 at E = 0 where that is a level
    assert np.all(np.diff(lnP[ks]) < 0)
    if (-eb) % 4 == 0:
        assert lnP[(-eb) // 4] == 0.0 or abs(lnP[(-eb) // 4]) < 1e-15
    # the enhancement at the ground state is Eq. (6): (1/(1 - E_g/dE))^alpha
    assert abs(lnP[k_lo] - alpha * math.log(1.0 / (1.0 - E_g / dE))) < 1e-12 * abs(lnP[k_lo]) + 1e-15


def test_rec_weights_invk_is_eq7(orc, exact_case):
    """The 1/k profile against Eq. (7) written out from integer counts: with S = ln g + c,
    ln P = ln g(k) - ln sum_{j=k_lo..k} g(j) and ln W = -S + ln P = -ln sum_{j<=k} g(j) + c'."""
    L, J, g, eb, k_lo, k_top = exact_case
    K = len(g)
    b = _exact_steps(g, k_lo, k_top)
    S, lnP, lnW = orc.rec_weights(K, eb, k_lo, k_top, 2, 1.0, 0.0, b)
    ks = np.arange(k_lo, k_top + 1)
    cum = np.cumsum([int(g[k]) for k in ks], dtype=object)          # exact integers
    ref_lnP = np.array([math.log(int(g[k])) - math.log(int(c)) for k, c in zip(ks, cum)])
    ref_lnW = np.array([math.log(int(g[k_top])) - math.log(int(c)) for c in cum])
    assert np.max(np.abs(lnP[ks] - ref_lnP)) <= 1e-12 * max(1.0, np.abs(ref_lnP).max())
    assert np.max(np.abs(lnW[ks] - ref_lnW)) <= 1e-12 * max(1.0, np.abs(ref_lnW).max())
    assert lnP[k_lo] == 0.0                                           # the ground state is all of its cumulative count
    assert np.all(lnP[ks] <= 1e-15)                                   # P = g / cumulative g <= 1
    assert np.all(np.diff(lnW[ks]) < 0)                               # W = 1/k falls with k
    # Sec. II: to first order the 1/k weights are a power law whose exponent is the slope of
    # ln g (P_SH ~ d ln g / dE); at the top, where ln g is nearly flat, the two agree best
    # (checked in ratio: the 1/k profile's local slope equals minus that of ln sum g)


@pytest.mark.parametrize("kind,dE,alpha", [("flat", 1.0, 0.0), ("power", 6.0, -2.0), ("invk", 1.0, 0.0)])
def test_production_from_exact_steps_gives_prescribed_histogram(orc, exact_L3, kind, dE, alpha):
    """Production (Sec. II) from a recursion state holding the exact steps: the oracle's own
    production weights must give H proportional to the prescribed distribution -- 1 (flat),
    P_SH of Eq. (5) anchored at the ground state (power law), g/sum_{E'<=E} g (1/k) -- each
    written out here from the enumerated counts."""
    L, J, g, = exact_L3
    eb, k_lo, k_top = _levels(orc, L, J, g)
    K = len(g)
    rz = orc.make_realization(L, 20110856, L3_REAL, 21, 48)
    st = orc.recursion_init(rz)
    st.b[:] = _exact_steps(g, k_lo, k_top)
    st.k_lo = k_lo
    lnw = orc.production_weights(rz, st, kind, pl_dE=dE, pl_alpha=alpha)
    H = _production_hist(orc, L, J, lnw[k_lo:k_top + 1], k_lo, k_top)
    ks = np.arange(k_lo, k_top + 1)
    E = eb + 4 * ks
    E_g = eb + 4 * k_lo
    if kind == "flat":
        target = np.ones(len(ks))
    elif kind == "power":
        target = ((E - E_g + dE) / (dE - E_g)) ** alpha
    else:
        gi = np.array([int(g[k]) for k in ks], dtype=np.float64)
        target = gi / np.cumsum(gi)
    h = H[ks] / H[ks].sum()
    p = target / target.sum()
    assert np.max(np.abs(h / p - 1)) < 0.12, (kind, np.c_[ks, h / p])
