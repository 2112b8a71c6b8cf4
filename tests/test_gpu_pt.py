"""GPU parity of parallel tempering (Sec. II, Eq. (8)) and of the round-trip statistics
(Sec. III) against the oracle.

With the same seeds and tables, spins, energies, minima, round-trip counters, slots,
exchange counters and energy traces agree bit for bit after PT sweeps (split launches,
L = 2..12, M = 8 and 32, mixed lattice sizes). Device-built tables agree with the
oracle's. tau per realization and tau_pop agree with the oracle's definition.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DSEED, WSEED = 20110856, 0x13572468


@pytest.fixture(scope="module")
def nfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_08560_amd import nfm as m
    m.lib()
    return m


def _bounds(L):
    # a configuration at T = 2 sits near E/N = -1.4, one at T = 0.2 near the ground state (-1.7 N)
    N = L ** 3
    return int(-1.6 * N), int(-1.45 * N)


def _run_pair(nfm, orc, Ls, W, M, n_sweeps, first=3, chunk=7, temps=None):
    T = orc.pt_temperatures(M)
    b = nfm.Batch(Ls, [W] * len(Ls), DSEED, WSEED, first_real_id=first, trace_capacity=n_sweeps)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    b.pt_init(T)
    if temps is not None:
        for r, Tr in enumerate(temps):
            b.pt_set_temps(r, Tr)
    for r, L in enumerate(Ls):
        e_bot, e_top = _bounds(L)
        b.set_rt_bounds(r, e_bot, e_top)
    b.set_tuning(sweeps_per_launch=chunk)
    b.pt_run_sweeps(n_sweeps // 2)
    b.pt_run_sweeps(n_sweeps - n_sweeps // 2)
    return b, T


def _tables_equal(nfm_tables, ref_metro, ref_swap):
    """The thresholds the kernel uses against the oracle's, bit for bit: the Metropolis rows are
    FP64 exp of the same arguments on both sides (the library's host code), the exchange
    thresholds q^d by the same binary powering (FP64 products, on the device and in the
    oracle) of the same q; the widths agree."""
    metro, swap = nfm_tables
    assert metro.shape == ref_metro.shape and swap.shape == ref_swap.shape
    assert np.array_equal(metro, ref_metro)
    assert np.array_equal(swap, ref_swap)


def _compare(nfm, orc, b, Ls, W, M, n_sweeps, temps, first=3, t0=0, states=None):
    """Every set of every realization against the oracle run from its initial state (or from
    `states`, the oracle's sets after an earlier run) over sweeps t0 .. t0 + n_sweeps."""
    ws = b.read_walkers()
    slots = b.pt_slots()
    acc = b.pt_exchanges(M)
    tr = b.read_trace()
    spw, sets_r = 64 // M, (W // 64) * (64 // M)
    out = {}
    for r, L in enumerate(Ls):
        N = L ** 3
        e_bot, e_top = _bounds(L)
        w0 = b.walker_offset(r)
        S_dev = b.get_spins(w0, W).reshape(W, N)
        Tr = temps[r]
        metro, swap = orc.pt_metro_table(Tr), orc.pt_swap_table(Tr, 3 * N // 2 + 1)
        for g in range(sets_r):
            ps = states[(r, g)] if states else orc.make_pt_set(L, DSEED, first + r, WSEED, M, set_index=g)
            a_ref = np.zeros(M - 1, np.uint64)
            tr_ref = orc.pt_sweeps(ps, metro, swap, e_bot, e_top, n_sweeps, swap_acc=a_ref, trace=True)
            k0 = ps.walker0
            sl = slice(w0 + k0, w0 + k0 + M)
            assert np.array_equal(S_dev[k0:k0 + M], ps.S), (L, r, g, "spins")
            for f in ("E", "E_min", "rt_state", "new_min", "rt_count", "t_first", "t_last"):
                assert np.array_equal(ws[f][sl], ps.w[f]), (L, r, g, f)
            assert np.array_equal(slots[sl], ps.slot), (L, r, g, "slots")
            assert np.array_equal(acc[r * sets_r + g], a_ref), (L, r, g, "exchanges")
            if tr is not None and tr.shape[1] >= t0 + n_sweeps:
                assert np.array_equal(tr[sl, t0:t0 + n_sweeps], tr_ref), (L, r, g, "trace")
            out[(r, g)] = ps
        # idle walkers of each group of 64: slot 0, no round-trip bookkeeping
        for q in range(W // 64):
            idle = slice(w0 + 64 * q + spw * M, w0 + 64 * (q + 1))
            assert np.all(slots[idle] == 0) and np.all(ws["rt_count"][idle] == 0)
    return out


@pytest.mark.parametrize("L,M,n", [(2, 32, 240), (4, 32, 160), (4, 8, 160), (6, 32, 60), (8, 32, 30),
                                   (10, 16, 16), (12, 32, 10), (4, 7, 120), (6, 14, 50), (8, 20, 24),
                                   (4, 12, 80)])
def test_pt_bit_exact(nfm, orc, L, M, n):
    Ls, W = [L, L], 64
    b, T = _run_pair(nfm, orc, Ls, W, M, n)
    _tables_equal(b.pt_tables(1), orc.pt_metro_table(T), orc.pt_swap_table(T, 3 * L ** 3 // 2 + 1))
    _compare(nfm, orc, b, Ls, W, M, n, [T, T])
    b.close()


def test_pt_mixed_sizes(nfm, orc):
    Ls, W, M, n = [4, 6, 4], 64, 16, 40
    b, T = _run_pair(nfm, orc, Ls, W, M, n, first=11)
    # the exchange thresholds are the same function of T for every L (their width D is where all vanish)
    _tables_equal(b.pt_tables(0), orc.pt_metro_table(T), orc.pt_swap_table(T, 3 * 6 ** 3 // 2 + 1))
    _compare(nfm, orc, b, Ls, W, M, n, [T] * 3, first=11)
    b.close()


def test_pt_per_realization_temperatures(nfm, orc):
    Ls, W, M, n = [4, 4, 6], 128, 12, 60
    temps = [orc.pt_temperatures(M, 0.2, 2.0), orc.pt_temperatures(M, 0.3, 3.2), orc.pt_temperatures(M, 0.25, 3.5)]
    b, _ = _run_pair(nfm, orc, Ls, W, M, n, first=21, temps=temps)
    for r in range(3):
        assert np.allclose(b.pt_temps(r, M), temps[r], rtol=1e-15, atol=0)
        _tables_equal(b.pt_tables(r), orc.pt_metro_table(temps[r]), orc.pt_swap_table(temps[r], 3 * Ls[r] ** 3 // 2 + 1))
    _compare(nfm, orc, b, Ls, W, M, n, temps, first=21)
    b.close()


def test_pt_adaptation_matches_oracle(nfm, orc):
    """Rates since the last step, the new temperatures of every realization, and the sweeps that
    follow under them."""
    Ls, W, M, n1, n2 = [4, 4], 64, 7, 60, 40
    b, T = _run_pair(nfm, orc, Ls, W, M, n1, first=31, chunk=1000)
    states = _compare(nfm, orc, b, Ls, W, M, n1, [T, T], first=31)
    acc = b.pt_exchanges(M)
    sets_r = 64 // M
    rates, n_out = b.pt_adapt(M, 0.4, 0.6)
    new_T = []
    for r in range(2):
        want = orc.pt_exchange_rates(acc[r * sets_r:(r + 1) * sets_r], 0, n1, M)
        assert np.allclose(rates[r], want, rtol=1e-15, atol=0)
        new_T.append(orc.pt_adapt_step(T, want))
        assert np.allclose(b.pt_temps(r, M), new_T[r], rtol=1e-12, atol=0)
    assert n_out == int(np.sum((rates < 0.4) | (rates > 0.6)))
    assert not np.any(b.pt_exchanges(M))                 # counters cleared
    b.pt_run_sweeps(n2)
    temps = [b.pt_temps(r, M) for r in range(2)]
    _compare(nfm, orc, b, Ls, W, M, n2, temps, first=31, t0=n1, states=states)
    b.close()


def test_pt_invalid_arguments(nfm):
    b = nfm.Batch([4], [64], DSEED, WSEED)
    with pytest.raises(nfm.NfmError):
        b.pt_init([0.5, 1.0])            # couplings not set
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    for T in ([1.0], [2.0, 1.0], [0.0, 1.0], [1.0] * 4, list(np.linspace(0.5, 3.0, 65))):
        with pytest.raises(nfm.NfmError):
            b.pt_init(T)
    with pytest.raises(nfm.NfmError):
        b.pt_run_sweeps(1)               # not initialised
    b.pt_init([0.5, 1.0, 2.0, 4.0])
    bad = np.zeros(64, np.int32)
    with pytest.raises(nfm.NfmError):
        b.pt_set_slots(bad)              # not a permutation per set
    ok = np.tile(np.array([3, 2, 1, 0], np.int32), 16)
    b.pt_set_slots(ok)
    assert np.array_equal(b.pt_slots(), ok)
    b.close()


def test_rt_stats_matches_oracle(nfm, orc):
    """Round trips from a PT run at L = 4, then tau per realization and
    tau_pop on the device against the oracle's definition on the same integer counters."""
    Ls, W, M, n = [4] * 6, 64, 8, 400
    T = orc.pt_temperatures(M)
    b = nfm.Batch(Ls, [W] * len(Ls), DSEED, WSEED, first_real_id=40)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    b.pt_init(T)
    for r in range(len(Ls)):
        b.set_rt_bounds(r, *_bounds(4))
    b.pt_run_sweeps(n)
    ws = b.read_walkers()
    for min_trips in (1, 40, 10 ** 9):
        tau, summ = b.rt_stats(0, len(Ls), min_trips=min_trips)
        ref = []
        for r in range(len(Ls)):
            sl = slice(r * W, (r + 1) * W)
            t_ref, trips, cens = orc.rt_tau(ws["rt_count"][sl], ws["t_first"][sl], ws["t_last"][sl], 64, min_trips)
            ref.append(t_ref)
            if cens:
                assert math.isnan(tau[r])
            else:
                assert abs(tau[r] - t_ref) <= 1e-14 * t_ref
        pop = orc.rt_population(ref)
        if math.isnan(pop):
            assert math.isnan(summ["tau_pop"]) and summ["n_used"] == 0
        else:
            assert abs(summ["tau_pop"] - pop) <= 1e-12 * pop
        assert summ["n_used"] + summ["n_censored"] == len(Ls)
        assert summ["trips"] == int(ws["rt_count"].sum())
    assert summ["n_censored"] == len(Ls)
    tau, summ = b.rt_stats(0, len(Ls), min_trips=1)
    assert summ["trips"] > 0, "the run must produce round trips for the check to mean anything"
    b.close()
