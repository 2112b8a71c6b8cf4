"""Pins for the oracle's parallel tempering (Sec. II, Eq. (8)) and its round-trip
statistics (Sec. III).

Independent facts used:
  * the stationary law of PT is the product of canonical laws, so at L = 2 the mean
    energy seen at every temperature slot matches the exact canonical mean from the
    enumerated density of states, and the exchange acceptance of every pair matches
    the exact mean of min(1, exp((1/T' - 1/T)(E' - E))) under the two canonical laws;
  * with temperatures that differ by 1e-15 every exchange succeeds, so the slot
    permutation after n sweeps is the product of the alternating transpositions and
    every pair's acceptance count equals the number of sweeps of its parity; with
    temperatures far apart only downhill exchanges succeed;
  * the incremental energy equals a recomputation after every sweep;
  * a hand-worked round-trip example (stamps fed through the tracker) gives the
    pooled tau of the definition.
"""
import math

import numpy as np
import pytest

DSEED, WSEED = 777, 0x5EED


def _exact_canonical(g, eb, T):
    E = eb + 4 * np.arange(len(g), dtype=np.float64)
    m = g > 0
    E, gg = E[m], g[m].astype(np.float64)
    lw = np.log(gg) - E / T
    p = np.exp(lw - lw.max())
    p /= p.sum()
    return E, p


def test_pt_canonical_means_and_exchange_rates_L2(orc):
    L, M = 2, 4
    T = np.array([0.6, 1.0, 1.7, 3.0])
    metro = orc.pt_metro_table(T)
    swap = orc.pt_swap_table(T, 3 * L ** 3 // 2 + 1)
    J = orc.couplings(L, DSEED, 3)
    g = orc.brute_dos(L, J)
    eb = orc.e_base(L, J)
    ps = orc.make_pt_set(L, DSEED, 3, WSEED, M)
    acc = np.zeros(M - 1, np.uint64)
    orc.pt_sweeps(ps, metro, swap, -10 ** 6, 10 ** 6, 2000)            # burn-in
    n, nb = 120_000, 40
    acc[:] = 0
    t_start = ps.t
    sums = np.zeros((nb, M))
    cnts = np.zeros((nb, M))
    for k in range(n):
        slot_before = ps.slot.copy()
        orc.pt_sweeps(ps, metro, swap, -10 ** 6, 10 ** 6, 1, swap_acc=acc)
        b = k * nb // n
        for c in range(M):
            sums[b, slot_before[c]] += ps.w["E"][c]
            cnts[b, slot_before[c]] += 1
    means = sums / cnts
    for s in range(M):
        E, p = _exact_canonical(g, eb, T[s])
        exact = float((E * p).sum())
        got = means[:, s].mean()
        err = means[:, s].std(ddof=1) / math.sqrt(nb)
        assert abs(got - exact) < 5 * err + 1e-9, (s, got, exact, err)
    # exchange acceptance per pair against the exact product-canonical expectation
    for s in range(M - 1):
        E0, p0 = _exact_canonical(g, eb, T[s])
        E1, p1 = _exact_canonical(g, eb, T[s + 1])
        db = 1.0 / T[s + 1] - 1.0 / T[s]
        x = np.minimum(1.0, np.exp(db * (E1[None, :] - E0[:, None])))
        exact = float((p0[:, None] * p1[None, :] * x).sum())
        tries = sum(1 for t in range(t_start, t_start + n) if t % 2 == s % 2)
        rate = acc[s] / tries
        assert abs(rate - exact) < 0.01, (s, rate, exact)


def test_pt_all_exchanges_when_temperatures_coincide(orc):
    L, M = 4, 6
    T = 1.0 + 1e-15 * np.arange(M)
    metro = orc.pt_metro_table(T)
    swap = orc.pt_swap_table(T, 3 * L ** 3 // 2 + 1)
    assert (swap == 0xFFFFFFFF).all()
    ps = orc.make_pt_set(L, DSEED, 1, WSEED, M, set_index=1)
    ps.t = 5                                     # odd start: pairs (1,2), (3,4) first
    acc = np.zeros(M - 1, np.uint64)
    n = 7
    orc.pt_sweeps(ps, metro, swap, -10 ** 6, 10 ** 6, n, swap_acc=acc, check_energy=True)
    at = list(range(M))                          # at[s] = configuration at slot s
    for t in range(5, 5 + n):
        for s in range(t % 2, M - 1, 2):
            at[s], at[s + 1] = at[s + 1], at[s]
    slot = np.empty(M, np.int32)
    for s, c in enumerate(at):
        slot[c] = s
    assert np.array_equal(ps.slot, slot)
    for s in range(M - 1):
        assert acc[s] == sum(1 for t in range(5, 5 + n) if t % 2 == s % 2)


def test_pt_far_temperatures_only_downhill_exchanges(orc):
    L, M = 4, 2
    T = np.array([0.05, 50.0])
    metro = orc.pt_metro_table(T)
    swap = orc.pt_swap_table(T, 3 * L ** 3 // 2 + 1)
    assert swap.shape[1] == 1 and swap[0, 0] == 0    # d = 1 already impossible
    ps = orc.make_pt_set(L, DSEED, 2, WSEED, M)
    for _ in range(200):
        before = ps.slot.copy()
        at = np.argsort(before)
        orc.pt_sweeps(ps, metro, swap, -10 ** 6, 10 ** 6, 1, check_energy=True)
        swapped = not np.array_equal(before, ps.slot)
        t = ps.t - 1
        if t % 2 == 0:
            d = (int(ps.w["E"][at[1]]) - int(ps.w["E"][at[0]])) // 4
            assert swapped == (d <= 0)
        else:
            assert not swapped


def test_pt_energy_consistency_and_tracking(orc):
    L, M = 4, 8
    T = orc.pt_temperatures(M)
    metro = orc.pt_metro_table(T)
    swap = orc.pt_swap_table(T, 3 * L ** 3 // 2 + 1)
    ps = orc.make_pt_set(L, DSEED, 4, WSEED, M)
    tr = orc.pt_sweeps(ps, metro, swap, -80, -40, 300, trace=True, check_energy=True)
    for c in range(M):
        assert ps.w["E_min"][c] == tr[c].min()
        assert ps.w["E"][c] == tr[c, -1]
        # round trips replayed from the trace with sweep-end stamps
        w = orc.new_walkers(1, 0)
        w["E_min"] = 10 ** 6
        for k in range(300):
            orc.track(w, int(tr[c, k]), -80, -40, (k + 1) * L ** 3)
        for f in ("rt_count", "t_first", "t_last", "rt_state"):
            assert w[f][0] == ps.w[f][c], (c, f)


def test_rt_tau_hand_example(orc):
    """Walker A: top at stamp 16, bottom, top at 96 (trip 1), bottom, top at 176 (trip 2);
    walker B: top at 40, bottom, top at 200 (trip 3); walker C never returns. N = 8:
    tau = ((176 - 16) + (200 - 40)) / 3 / 8 = 13.333.. sweeps."""
    N, e_bot, e_top = 8, -12, 0
    w = orc.new_walkers(3, -4)
    w["E_min"] = -4
    seq = {0: [(16, 0), (50, -12), (96, 0), (120, -16), (176, 4)],
           1: [(40, 0), (100, -12), (200, 0)],
           2: [(8, 0), (9, -12)]}
    for k, events in seq.items():
        one = w[k:k + 1].copy()
        for tau, E in events:
            orc.track(one, E, e_bot, e_top, tau)
        w[k] = one[0]
    assert list(w["rt_count"]) == [2, 1, 0]
    assert w["new_min"][0] == 1 and w["new_min"][1] == 0
    tau, trips, cens = orc.rt_tau(w["rt_count"], w["t_first"], w["t_last"], N)
    assert trips == 3 and not cens
    assert abs(tau - 320 / 3 / 8) < 1e-12
    tau, trips, cens = orc.rt_tau(w["rt_count"], w["t_first"], w["t_last"], N, min_trips=4)
    assert cens and math.isnan(tau)
    assert orc.rt_population([1.0, float("nan"), 3.0]) == 2.0


# ----------------------------------------------------------------------------- temperature adaptation

def test_pt_set_walkers_fill_groups_of_64(orc):
    # floor(64/M) sets per group of 64 walkers, the rest of the group idle
    assert [orc.pt_set_walker0(7, g) for g in range(11)] == [0, 7, 14, 21, 28, 35, 42, 49, 56, 64, 71]
    assert [orc.pt_set_walker0(20, g) for g in range(5)] == [0, 20, 40, 64, 84]
    assert [orc.pt_set_walker0(32, g) for g in range(4)] == [0, 32, 64, 96]


def test_exchange_rates_count_attempts_by_parity(orc):
    acc = np.array([[3, 4, 5], [1, 2, 3]])
    # sweeps 5..10: t = 5, 7, 9 attempt odd pairs (s = 1), t = 6, 8, 10 even ones (s = 0, 2)
    r = orc.pt_exchange_rates(acc, 5, 11, 4)
    assert np.allclose(r, [4 / 6, 6 / 6, 8 / 6])
    r = orc.pt_exchange_rates(acc, 5, 10, 4)   # t = 6, 8 even; 5, 7, 9 odd
    assert np.allclose(r, [4 / 4, 6 / 6, 8 / 4])


def test_adapt_step_fixed_point_and_ends(orc):
    T = orc.pt_temperatures(9, 0.2, 3.2)
    same = orc.pt_adapt_step(T, np.full(8, 0.37))
    assert np.allclose(same, T, rtol=1e-14, atol=0)
    new = orc.pt_adapt_step(T, np.array([0.5, 0.5, 0.1, 0.5, 0.5, 0.5, 0.9, 0.5]))
    assert new[0] == T[0] and new[-1] == pytest.approx(T[-1], rel=1e-15)
    assert np.all(np.diff(new) > 0)
    g_old, g_new = np.diff(1 / T), np.diff(1 / new)
    # the pair with the fewest exchanges gets a narrower gap, the one with the most a wider one
    ratio = g_new / g_old
    assert ratio[2] < ratio[0] < ratio[6]


def test_adapt_step_factor_is_limited(orc):
    # a pair that always exchanges (A = 1: both temperatures in the ground state) widens by 2 (not
    # by (1e-12)^(-1/4) = 1000), one that never does narrows by (-ln 1e-6)^(-1/4), before the gaps
    # are rescaled to their old sum
    T = orc.pt_temperatures(4, 0.2, 3.2)
    new = orc.pt_adapt_step(T, np.array([1.0, 0.0, np.exp(-1.0)]))
    g_old, g_new = np.diff(1 / T), np.diff(1 / new)
    k = g_new[2] / g_old[2]          # the pair with -ln A = 1 keeps its factor 1: k is the rescale
    assert g_new[0] / g_old[0] == pytest.approx(2.0 * k, rel=1e-13)
    assert g_new[1] / g_old[1] == pytest.approx(math.log(1e6) ** -0.25 * k, rel=1e-13)
    assert np.sum(g_new) == pytest.approx(np.sum(g_old), rel=1e-14)


def test_adapt_converges_to_equal_rates_on_a_gaussian_model(orc):
    # overlapping Gaussian energy distributions: A_s = exp(-c_s gap_s^2), c_s growing toward low T
    M = 12
    T = orc.pt_temperatures(M, 0.2, 3.2)
    c = np.linspace(10.0, 1.0, M - 1)
    for _ in range(80):
        gaps = np.diff(-1.0 / T)          # beta_s - beta_{s+1} > 0
        T = orc.pt_adapt_step(T, np.exp(-c * gaps ** 2))
    A = np.exp(-c * np.diff(-1.0 / T) ** 2)
    assert A.max() - A.min() < 1e-6 * A.mean()
    assert T[0] == pytest.approx(0.2, rel=1e-14) and T[-1] == pytest.approx(3.2, rel=1e-12)


def test_swap_probability_by_binary_powering(orc):
    """q^d by binary powering equals exp(d ln q) to rounding, and exp(4 d (1/T_hi - 1/T_lo))
    (Eq. (8)) to a few units in the last place; the table quantizes exactly these values."""
    import math
    T = orc.pt_temperatures(8, 0.2, 3.2)
    q = orc.pt_swap_q(T[2], T[3])
    assert q == math.exp(4.0 * (1.0 / T[3] - 1.0 / T[2]))
    for d in (1, 2, 3, 7, 64, 100, 1023):
        assert orc.pow_bin(q, d) == pytest.approx(math.exp(4.0 * d * (1.0 / T[3] - 1.0 / T[2])), rel=1e-13)
    r = 1.0
    for d in range(1, 40):          # repeated products agree with the powering to rounding
        r *= q
        assert orc.pow_bin(q, d) == pytest.approx(r, rel=1e-14)
    tab = orc.pt_swap_table(T, 200)
    assert tab[2, 6] == math.floor(math.ldexp(orc.pow_bin(q, 7), 32))
    assert np.all(np.diff(tab.astype(np.int64), axis=1) <= 0)
