"""Pins for the oracle's Markov chain (Eq. (2)), threshold tables and round-trip
bookkeeping (Sec. III).

Independent facts used:
  * all-accept tables flip every spin once per sweep (S -> -S, E unchanged);
    all-reject tables freeze the state;
  * at L = 2 the exact 256-state transition matrix of one sweep, built here
    from the definition of the chain, gives the exact distribution after T
    sweeps; the oracle's walkers are chi-square tested against it, and the
    stationary vector is proportional to W up to the 2^-32 quantization;
  * with canonical weights W = exp(-beta E) the sampled mean energy at L = 3
    matches the exact value from the enumerated density of states;
  * thresholds of canonical weights have the closed form floor(exp(-beta dE) 2^32);
  * a compact table with clamped rows equals the full-range table;
  * Eq. (6): the power-law profile at E_g (golden values of the paper).
"""
import itertools
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FULL = 0xFFFFFFFF


def _canonical_lnw(eb, k_lo, k_top, beta):
    E = eb + 4 * np.arange(k_lo, k_top + 1)
    return -beta * E.astype(np.float64)


def _all_accept_table(rows):
    return np.full((rows, 8), FULL, np.uint32)


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_all_accept_flips_every_spin(orc, L):
    J = orc.couplings(L, 3, 1)
    S = orc.spins(L, 4, 1, 0)
    E0 = orc.energy(L, J, S)
    w = orc.new_walkers(1, E0)
    K = orc.n_levels(L, J)
    S1 = S.copy()
    orc.muca_sweeps(L, J, S1, w, _all_accept_table(K), 0, -10 ** 6, 10 ** 6, 9, 1, 0, 0, 1, check_energy=True)
    assert np.array_equal(S1, -S)
    assert w["E"][0] == E0
    orc.muca_sweeps(L, J, S1, w, np.zeros((K, 8), np.uint32), 0, -10 ** 6, 10 ** 6, 9, 1, 0, 1, 3)
    assert np.array_equal(S1, -S)


def test_incremental_energy_matches_recomputation(orc):
    rng = np.random.default_rng(3)
    for L in (2, 3, 4, 6):
        J = orc.couplings(L, 8, 2)
        K, eb = orc.n_levels(L, J), orc.e_base(L, J)
        lnw = np.cumsum(rng.normal(0.3, 1.0, K))
        thr, row0 = orc.build_thresholds(K, lnw, 0, K - 1)
        S = orc.spins(L, 1, 2, 0)
        w = orc.new_walkers(1, orc.energy(L, J, S))
        orc.muca_sweeps(L, J, S, w, thr, row0, -10 ** 6, 10 ** 6, 5, 2, 0, 0, 20, check_energy=True)


# ----------------------------------------------------------------------------- L = 2 exact chain

def _state_spins(s, N):
    return np.array([-1 if (s >> i) & 1 else 1 for i in range(N)], np.int8)


def _exact_sweep_matrix(L, J, thr, row0):
    """Row-stochastic matrix of one sweep, from the chain's definition: sites in
    checkerboard order; at each site flip with probability thr/2^32 (1 if
    0xFFFFFFFF) where thr is the entry of the (clamped) row of the current level
    and the number u of unsatisfied bonds."""
    N = L ** 3
    eb = -3 * N + 2 * (int((J < 0).sum()) % 2)
    nS = 2 ** N
    Es = np.zeros(nS, np.int64)
    U = np.zeros((nS, N), np.int64)
    coords = [(i % L, (i // L) % L, i // (L * L)) for i in range(N)]
    idx = lambda x, y, z: (x % L) + L * (y % L) + L * L * (z % L)
    for s in range(nS):
        S = _state_spins(s, N).astype(np.int64)
        e = 0
        for i, (x, y, z) in enumerate(coords):
            for d, (dx, dy, dz) in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
                j = idx(x + dx, y + dy, z + dz)
                e -= J[d * N + i] * S[i] * S[j]
                # bond (i, j) unsatisfied <=> J S_i S_j = -1; it touches both ends
                if J[d * N + i] * S[i] * S[j] < 0:
                    U[s, i] += 1
                    U[s, j] += 1
        Es[s] = e
    order = [i for c in (0, 1) for i in range(N) if sum(coords[i]) % 2 == c]
    rows = thr.shape[0]
    M = np.eye(nS)
    for i in order:
        T = np.zeros((nS, nS))
        for s in range(nS):
            k = (Es[s] - eb) // 4
            r = min(max(k - row0, 0), rows - 1)
            th = int(thr[r, U[s, i]])
            p = 1.0 if th == FULL else max(th, 1) / 2.0 ** 32
            T[s, s ^ (1 << i)] += p
            T[s, s] += 1.0 - p
        M = M @ T
    return M, Es, eb


def test_exact_chain_L2(orc):
    L, N = 2, 8
    J = orc.couplings(L, 20110856, 3)
    K, eb = orc.n_levels(L, J), orc.e_base(L, J)
    rng = np.random.default_rng(11)
    lnw = np.cumsum(rng.normal(0.4, 0.6, K))      # generic, non-canonical weights
    thr, row0 = orc.build_thresholds(K, lnw, 0, K - 1)
    M, Es, _ = _exact_sweep_matrix(L, J, thr, row0)
    assert np.allclose(M.sum(axis=1), 1.0)
    # W(E) is left invariant by every single-site step (detailed balance), hence
    # by the sweep, up to the 2^-32 quantization of the acceptances. (Tiny
    # lattices can have several closed classes, so test invariance, not uniqueness.)
    Wst = np.exp(lnw[(Es - eb) // 4] - lnw.max())
    Wst /= Wst.sum()
    assert np.max(np.abs((Wst @ M) / Wst - 1.0)) < 1e-6
    # oracle walkers started from one state: distribution after T sweeps = e_s0 M^T
    s0, T, nw = 5, 3, 6000
    exact = np.linalg.matrix_power(M, T)[s0]
    counts = np.zeros(2 ** N)
    S0 = _state_spins(s0, N)
    for wk in range(nw):
        S = S0.copy()
        w = orc.new_walkers(1, orc.energy(L, J, S))
        orc.muca_sweeps(L, J, S, w, thr, row0, -10 ** 6, 10 ** 6, 0xC0FFEE, 3, wk, 0, T)
        counts[int(sum(1 << i for i in range(N) if S[i] < 0))] += 1
    exp = exact * nw
    big = exp >= 5
    chi2 = (((counts[big] - exp[big]) ** 2) / exp[big]).sum() + \
        ((counts[~big].sum() - exp[~big].sum()) ** 2) / max(exp[~big].sum(), 1e-9)
    dof = int(big.sum())
    # p ~ 1e-4 bound for chi-square with dof degrees of freedom (Wilson-Hilferty)
    bound = dof * (1 - 2 / (9 * dof) + 3.72 * math.sqrt(2 / (9 * dof))) ** 3
    assert chi2 < bound, (chi2, dof)
    assert counts[exp == 0].sum() == 0


def test_canonical_mean_energy_L3(orc):
    L, N, beta = 3, 27, 0.35
    J = orc.couplings(L, 20110856, 0)
    g = orc.brute_dos(L, J).astype(np.float64)
    K, eb = orc.n_levels(L, J), orc.e_base(L, J)
    E = eb + 4 * np.arange(K)
    m = g > 0
    a = np.log(g[m]) - beta * E[m]
    p = np.exp(a - a.max())
    exact = float((p * E[m]).sum() / p.sum())
    thr, row0 = orc.build_thresholds(K, _canonical_lnw(eb, 0, K - 1, beta), 0, K - 1)
    nw, burn, ns = 24, 100, 1500
    means = []
    for wk in range(nw):
        S = orc.spins(L, 2, 0, wk)
        w = orc.new_walkers(1, orc.energy(L, J, S))
        orc.muca_sweeps(L, J, S, w, thr, row0, -10 ** 6, 10 ** 6, 13, 0, wk, 0, burn)
        tr = np.zeros(ns, np.int32)
        orc.muca_sweeps(L, J, S, w, thr, row0, -10 ** 6, 10 ** 6, 13, 0, wk, burn, ns, trace=tr)
        means.append(tr.mean())
    means = np.array(means)
    err = means.std(ddof=1) / math.sqrt(nw)
    assert abs(means.mean() - exact) < 5 * err + 1e-9, (means.mean(), exact, err)


# ----------------------------------------------------------------------------- thresholds

def test_thresholds_canonical_closed_form(orc):
    L, beta = 4, 0.7
    J = orc.couplings(L, 1, 0)
    K, eb = orc.n_levels(L, J), orc.e_base(L, J)
    thr, row0 = orc.build_thresholds(K, _canonical_lnw(eb, 0, K - 1, beta), 0, K - 1)
    assert row0 == 0
    for k in range(3, K - 3):
        for u in range(7):
            dE = 12 - 4 * u
            if dE <= 0:
                assert thr[k, u] == FULL
            else:
                ref = math.floor(math.exp(-beta * dE) * 2 ** 32)
                assert abs(int(thr[k, u]) - ref) <= 1
        assert thr[k, 7] == 0


def _full_row(lnw, k_lo, k_top, k):
    """Entry values of row k from the definition (step log-weights with the
    continuation rules), without clamping."""
    def d(j):
        j = max(j, k_lo)
        if j >= k_top:
            return 0.0
        return lnw[j + 1 - k_lo] - lnw[j - k_lo]
    out = []
    for u in range(7):
        m = 3 - u
        if m == 0:
            x = 1.0
        elif m > 0:
            s = 0.0
            for j in range(k, k + m):
                s += d(j)
            x = math.exp(s)
        else:
            s = 0.0
            for j in range(k + m, k):
                s += d(j)
            x = math.exp(-s)
        out.append((FULL if x >= 1.0 else math.floor(math.ldexp(x, 32)), x))
    return out


def test_compact_table_with_clamps_equals_full_table(orc):
    rng = np.random.default_rng(5)
    L = 4
    J = orc.couplings(L, 1, 4)
    K = orc.n_levels(L, J)
    for k_lo, k_top in ((10, 48), (0, 48), (40, K - 1), (5, 5), (30, 31)):
        lnw = np.cumsum(rng.normal(-0.5, 1.5, k_top - k_lo + 1))
        thr, row0 = orc.build_thresholds(K, lnw, k_lo, k_top)
        assert row0 == max(0, k_lo - 3)
        assert thr.shape[0] == min(K - 1, k_top + 3) - row0 + 1
        for k in range(K):
            r = min(max(k - row0, 0), thr.shape[0] - 1)
            for u, (ref, x) in enumerate(_full_row(lnw, k_lo, k_top, k)):
                got = int(thr[r, u])
                if got != ref:
                    # only where exp's last bit decides the floor
                    assert abs(got - ref) == 1 and abs(math.ldexp(x, 32) - round(math.ldexp(x, 32))) < 1e-5


def test_power_profile_golden(orc):
    """Eq. (6): enhancement of P_SH at E_g relative to E = 0 (alpha=-3.6, dE=96)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "profile_enhancement.txt")) if l.strip() and not l.startswith("#")]
    for E_g, approx, rel in rows:
        E_g, approx, rel = float(E_g), float(approx), float(rel)
        v = orc.power_profile(E_g, E_g, 96.0, -3.6)
        closed = (1.0 / (1.0 - E_g / 96.0)) ** -3.6
        assert abs(v / closed - 1) < 1e-12
        assert abs(v / approx - 1) < rel
        assert orc.power_profile(0.0, E_g, 96.0, -3.6) == 1.0


# ----------------------------------------------------------------------------- round trips

def test_round_trip_tracker_synthetic(orc):
    e_bot, e_top = -40, 0
    # energies after successive attempts, hand-counted: tops at steps 2, 6, 10;
    # bottoms at 4 and 8 (the -44 at step 9 is below e_bot: new minimum).
    trace = [-8, 0, -20, -40, -12, 4, -36, -40, -44, 0, -40]
    w = orc.new_walkers(1, -8)
    for s, e in enumerate(trace, start=1):
        orc.track(w, e, e_bot, e_top, s)
    assert w["rt_count"][0] == 2
    assert w["t_first"][0] == 2
    assert w["t_last"][0] == 10
    assert w["E_min"][0] == -44
    assert w["new_min"][0] == 1
    assert w["rt_state"][0] == 2
    # bottom first, then top: no trip counted until bottom-after-top-then-top
    w = orc.new_walkers(1, -40)
    for s, e in enumerate([-40, -40, 0, -40, -4, 8], start=1):
        orc.track(w, e, e_bot, e_top, s)
    assert w["rt_count"][0] == 1 and w["t_first"][0] == 3 and w["t_last"][0] == 6
    assert w["new_min"][0] == 0


def test_acceptance_rule(orc):
    """Acceptance of an attempt: probability thr / 2^32 (r < thr for r uniform on 32 bits),
    always for the all-accept value, and never below 2^-32 (thr = 0 accepts r = 0 only)."""
    acc = orc.metropolis_accept
    assert acc(0, FULL) and acc(FULL, FULL) and acc(FULL - 1, FULL)
    assert acc(4, 5) and not acc(5, 5) and not acc(FULL, 5)
    assert acc(0, 1) and not acc(1, 1)
    assert acc(0, 0) and not acc(1, 0) and not acc(FULL, 0)
    assert acc(FULL - 2, FULL - 1) and not acc(FULL - 1, FULL - 1)


def test_acceptance_word_layout(orc):
    """With every threshold equal to 2^31 an attempt is accepted iff its random
    word is below 2^31, whatever the state, so one sweep flips exactly the sites
    whose word (re-derived here from the documented counter layout) is small."""
    for L in (2, 3, 4, 6):
        N = L ** 3
        J = orc.couplings(L, 1, 0)
        K = orc.n_levels(L, J)
        S0 = orc.spins(L, 2, 9, 3)
        S = S0.copy()
        w = orc.new_walkers(1, orc.energy(L, J, S))
        thr = np.full((K, 8), 2 ** 31, np.uint32)
        seed, t, real, walker = 0xDEADBEEF12345678, 7, 9, 3
        orc.muca_sweeps(L, J, S, w, thr, 0, -10 ** 6, 10 ** 6, seed, real, walker, t, 1)
        key = [seed & 0xFFFFFFFF, seed >> 32]
        for i in range(N):
            x, y, z = i % L, (i // L) % L, i // (L * L)
            c = (x + y + z) % 2
            q = sum(1 for yy in range(L) for xx in range(L) if (xx + yy + z) % 2 == c and xx + L * yy < x + L * y)
            r = orc.philox([((c * L + z) << 8) | (q >> 2), t, real, (walker << 8) | orc.TAG_ACC], key)[q & 3]
            assert (S[i] != S0[i]) == (int(r) < 2 ** 31)
