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


def _run_pair(nfm, orc, Ls, W, M, n_sweeps, first=3, chunk=7):
    T = orc.pt_temperatures(M)
    b = nfm.Batch(Ls, [W] * len(Ls), DSEED, WSEED, first_real_id=first, trace_capacity=n_sweeps)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    b.pt_init(T)
    metro, swap = b.pt_tables()
    for r, L in enumerate(Ls):
        e_bot, e_top = _bounds(L)
        b.set_rt_bounds(r, e_bot, e_top)
    b.set_tuning(sweeps_per_launch=chunk)
    b.pt_run_sweeps(n_sweeps // 2)
    b.pt_run_sweeps(n_sweeps - n_sweeps // 2)
    return b, T, metro, swap


def _compare(nfm, orc, b, Ls, W, M, n_sweeps, metro, swap, first=3):
    ws = b.read_walkers()
    slots = b.pt_slots()
    acc = b.pt_exchanges(M)
    tr = b.read_trace()
    assert tr.shape[1] == n_sweeps
    for r, L in enumerate(Ls):
        N = L ** 3
        e_bot, e_top = _bounds(L)
        w0 = b.walker_offset(r)
        S_dev = b.get_spins(w0, W).reshape(W, N)
        for g in range(W // M):
            ps = orc.make_pt_set(L, DSEED, first + r, WSEED, M, set_index=g)
            a_ref = np.zeros(M - 1, np.uint64)
            tr_ref = orc.pt_sweeps(ps, metro, swap, e_bot, e_top, n_sweeps, swap_acc=a_ref, trace=True)
            sl = slice(w0 + g * M, w0 + (g + 1) * M)
            assert np.array_equal(S_dev[g * M:(g + 1) * M], ps.S), (L, r, g, "spins")
            for f in ("E", "E_min", "rt_state", "new_min", "rt_count", "t_first", "t_last"):
                assert np.array_equal(ws[f][sl], ps.w[f]), (L, r, g, f)
            assert np.array_equal(slots[sl], ps.slot), (L, r, g, "slots")
            assert np.array_equal(acc[(w0 // M) + g], a_ref), (L, r, g, "exchanges")
            assert np.array_equal(tr[sl, :n_sweeps], tr_ref), (L, r, g, "trace")


@pytest.mark.parametrize("L,M,n", [(2, 32, 240), (4, 32, 160), (4, 8, 160), (6, 32, 60), (8, 32, 30),
                                   (10, 16, 16), (12, 32, 10)])
def test_pt_bit_exact(nfm, orc, L, M, n):
    Ls, W = [L, L], 64
    b, T, metro, swap = _run_pair(nfm, orc, Ls, W, M, n)
    ref_metro = orc.pt_metro_table(T)
    ref_swap = orc.pt_swap_table(T, 3 * L ** 3 // 2 + 1)
    assert np.array_equal(metro, ref_metro)
    assert np.array_equal(swap, ref_swap)
    _compare(nfm, orc, b, Ls, W, M, n, metro, swap)
    b.close()


def test_pt_mixed_sizes(nfm, orc):
    Ls, W, M, n = [4, 6, 4], 64, 16, 40
    b, T, metro, swap = _run_pair(nfm, orc, Ls, W, M, n, first=11)
    # the exchange table is the same function of T for every L (its width D is where all rows vanish)
    ref_swap = orc.pt_swap_table(T, 3 * 6 ** 3 // 2 + 1)
    assert np.array_equal(swap, ref_swap)
    _compare(nfm, orc, b, Ls, W, M, n, metro, swap, first=11)
    b.close()


def test_pt_invalid_arguments(nfm):
    b = nfm.Batch([4], [64], DSEED, WSEED)
    with pytest.raises(nfm.NfmError):
        b.pt_init([0.5, 1.0])            # couplings not set
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    for T in ([1.0, 2.0, 3.0], [2.0, 1.0], [0.0, 1.0], [1.0] * 4):
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
