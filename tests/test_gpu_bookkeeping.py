"""Exact bookkeeping with round-trip bounds two levels apart (Sec. III): walkers cross the bottom
and the top again and again, several times within one check interval of the sweep kernel (every
8 attempts at small L, 16 at L = 10, 32 at L = 12), so the ordered replay of the round-trip state
and the order-free minimum and new-minimum flag are all exercised. Every walker's minimum, flag,
state, trip count and first / last stamps must equal the oracle's, which tracks each attempt in
turn, for every kernel form the library picks (plain, speculative, persistent queue, split)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DSEED, WSEED = 20110856, 0xB00C
LS = [4, 6, 10, 12]
FIRST = 90


@pytest.fixture(scope="module")
def nfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_08560_amd import nfm as m
    m.lib()
    return m


def _tables(orc):
    out = []
    for r, L in enumerate(LS):
        J = orc.couplings(L, DSEED, FIRST + r)
        K, eb = orc.n_levels(L, J), orc.e_base(L, J)
        k_top = (-eb + 3) // 4
        k_lo = max(0, k_top - int(0.45 * L ** 3))
        lnw = -0.7 * (eb + 4 * np.arange(k_lo, k_top + 1, dtype=np.float64))
        thr, row0 = orc.build_thresholds(K, lnw, k_lo, k_top)
        out.append((thr, row0, eb + 4 * k_lo, eb))
    return out


FIELDS = ("E", "E_min", "rt_state", "new_min", "rt_count", "t_first", "t_last")


@pytest.mark.parametrize("tuning", [dict(schedule=0, speculate=0), dict(schedule=0, speculate=1),
                                    dict(schedule=1, speculate=0, sweeps_per_launch=7),
                                    dict(schedule=2, speculate=0, sweeps_per_launch=5)])
def test_close_bounds_match_oracle(nfm, orc, tuning):
    n1, n2 = 6, 14
    print("bookkeeping: close bounds", tuning, flush=True)
    tabs = _tables(orc)
    b = nfm.Batch(LS, [64] * len(LS), DSEED, WSEED, first_real_id=FIRST)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    for r, (thr, row0, e_bot, _) in enumerate(tabs):
        b.set_thresholds(r, thr, row0)
        b.set_rt_bounds(r, e_bot, 0)
    b.set_tuning(**tuning)
    b.run_sweeps(n1)
    ws = b.read_walkers()
    rzs = []
    for r, L in enumerate(LS):
        thr, row0, e_bot, eb = tabs[r]
        rz = orc.make_realization(L, DSEED, FIRST + r, WSEED, 64)
        orc.sample(rz, thr, row0, e_bot, 0, n1)
        rzs.append(rz)
    # bounds two levels apart around the walkers' median energy: crossings several times per check
    bounds = []
    for r, L in enumerate(LS):
        w0 = b.walker_offset(r)
        eb = tabs[r][3]
        e_mid = int(np.median(ws["E"][w0:w0 + 64]))
        e_top = eb + 4 * ((e_mid - eb) // 4)
        bounds.append((e_top - 8, e_top))
        b.set_rt_bounds(r, e_top - 8, e_top)
    b.run_sweeps(n2)
    ws = b.read_walkers()
    crossed = 0
    for r, L in enumerate(LS):
        thr, row0, _, _ = tabs[r]
        e_bot, e_top = bounds[r]
        orc.sample(rzs[r], thr, row0, e_bot, e_top, n2)
        w0 = b.walker_offset(r)
        for f in FIELDS:
            assert np.array_equal(ws[f][w0:w0 + 64], rzs[r].w[f]), (L, f)
        crossed += int(rzs[r].w["rt_count"].sum())
    assert crossed > 64 * len(LS) * 3, crossed      # many round trips: the replay did run
    b.close()
