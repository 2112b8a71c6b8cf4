"""Mixed-size batches: the persistent work-queue launch and the autotuner.

The launch configuration (per-size launches or one persistent launch, speculation, sweeps
per launch, workgroups per CU) must not change any result: spins, walker bookkeeping,
histograms and traces are compared bit for bit across configurations, and one realization
of every size against the oracle. The autotuner must leave the batch exactly as it found it.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DSEED, WSEED = 20110856, 0x2468ACE0
MIX = [12, 4, 6, 4, 8, 4, 10, 6, 4, 8, 4, 6, 4]


@pytest.fixture(scope="module")
def nfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_08560_amd import nfm as m
    m.lib()
    return m


def _tables(orc, Ls, first):
    out = []
    for r, L in enumerate(Ls):
        J = orc.couplings(L, DSEED, first + r)
        K, eb = orc.n_levels(L, J), orc.e_base(L, J)
        k_top = (-eb + 3) // 4
        k_lo = max(0, k_top - int(0.45 * L ** 3))
        lnw = -0.7 * (eb + 4 * np.arange(k_lo, k_top + 1, dtype=np.float64))
        out.append(orc.build_thresholds(K, lnw, k_lo, k_top) + (eb + 4 * k_lo,))
    return out


def _batch(nfm, orc, Ls, n_trace, first=5):
    b = nfm.Batch(Ls, [64] * len(Ls), DSEED, WSEED, first_real_id=first, trace_capacity=n_trace)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    for r, (thr, row0, e_bot) in enumerate(_tables(orc, Ls, first)):
        b.set_thresholds(r, thr, row0)
        b.set_rt_bounds(r, e_bot, 0)
    return b


def _state(b):
    return (b.get_spins(0, b.n_walkers), b.read_walkers(), b.read_histograms(), b.read_trace())


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_spins_roundtrip_across_sizes(nfm, orc):
    """One set/get call over walkers of realizations of different L."""
    b = nfm.Batch(MIX, [64] * len(MIX), DSEED, WSEED)
    rng = np.random.default_rng(5)
    total = sum(64 * L ** 3 for L in MIX)
    S = rng.choice(np.array([-1, 1], np.int8), total)
    b.set_spins(0, S)
    assert np.array_equal(b.get_spins(0, b.n_walkers), S)
    w0 = b.walker_offset(1) + 60                     # a range across the L=4 / L=6 boundary
    part = b.get_spins(w0, 10)
    lo = sum(64 * L ** 3 for L in MIX[:1]) + 60 * 64
    assert np.array_equal(part, S[lo:lo + 4 * 64 + 6 * 216])
    b.close()


# hist: 0 automatic, 1 window, 2 every level, 3 the table rows alone (most counts outside LDS)
CONFIGS = [dict(schedule=1, speculate=0, sweeps_per_launch=0, waves_per_cu=0, hist=0, ws=0),
           dict(schedule=1, speculate=1, sweeps_per_launch=7, waves_per_cu=0, hist=1, ws=0),
           dict(schedule=1, speculate=0, sweeps_per_launch=16, waves_per_cu=1, hist=3, ws=0),
           dict(schedule=1, speculate=1, sweeps_per_launch=0, waves_per_cu=3, hist=2, ws=0),
           dict(schedule=0, speculate=1, sweeps_per_launch=9, waves_per_cu=0, hist=3, ws=0),
           dict(schedule=0, speculate=0, sweeps_per_launch=11, waves_per_cu=0, hist=1, ws=0),
           dict(schedule=0, speculate=0, sweeps_per_launch=13, waves_per_cu=0, hist=0, ws=2),
           dict(schedule=0, speculate=0, sweeps_per_launch=0, waves_per_cu=0, hist=0, ws=1),
           # split: the largest size in the SIMD-exclusive form beside a queue over the others
           dict(schedule=2, speculate=0, sweeps_per_launch=0, waves_per_cu=0, hist=0, ws=0),
           dict(schedule=2, speculate=1, sweeps_per_launch=7, waves_per_cu=0, hist=1, ws=0),
           dict(schedule=2, speculate=0, sweeps_per_launch=16, waves_per_cu=0, hist=3, ws=0)]


def test_schedules_give_identical_results(nfm, orc):
    n = 40
    ref = _batch(nfm, orc, MIX, n)
    ref.set_tuning(schedule=0, speculate=0)
    ref.run_sweeps(n)
    want = _state(ref)
    ref.close()
    for cfg in CONFIGS:
        print("tuning", cfg, flush=True)
        b = _batch(nfm, orc, MIX, n)
        b.set_tuning(**cfg)
        assert b.get_tuning() == dict(cfg, sweeps_per_launch=cfg["sweeps_per_launch"] or 1024)
        b.run_sweeps(n // 3)
        b.run_sweeps(n - n // 3)
        if cfg["schedule"] == 2:
            assert b.last_kernel().endswith("_solo"), (b.last_kernel(), b._lib.nfm_last_error(b.ctx))
        _same(_state(b), want)
        b.close()


@pytest.mark.parametrize("schedule,hist", [(1, 0), (1, 3), (2, 0)])
def test_queue_matches_oracle(nfm, orc, schedule, hist):
    n, first = 24, 5
    b = _batch(nfm, orc, MIX, 0, first=first)
    b.set_tuning(schedule=schedule, speculate=1, sweeps_per_launch=10, hist=hist)
    b.run_sweeps(n)
    assert b.last_kernel() == ("k_sweeps_queue_spec" if schedule == 1 else "k_sweeps_queue_spec_solo")
    ws = b.read_walkers()
    H = b.read_histograms()
    tabs = _tables(orc, MIX, first)
    seen = set()
    for r, L in enumerate(MIX):
        if L in seen:
            continue
        seen.add(L)
        thr, row0, e_bot = tabs[r]
        rz = orc.make_realization(L, DSEED, first + r, WSEED, 64)
        Hr, _ = orc.sample(rz, thr, row0, e_bot, 0, n)
        off = b.level_offset(r)
        assert np.array_equal(H[off:off + rz.K], Hr), L
        w0 = b.walker_offset(r)
        assert np.array_equal(b.get_spins(w0, 64).reshape(64, -1), rz.S), L
        for f in ("E", "E_min", "rt_state", "new_min", "rt_count", "t_first", "t_last"):
            assert np.array_equal(ws[f][w0:w0 + 64], rz.w[f]), (L, f)
    b.close()


def test_autotune_restores_state_and_caches(nfm, orc, tmp_path):
    b = _batch(nfm, orc, MIX, 0)
    b.run_sweeps(10)
    before = _state(b)
    t_before = b.sweep_counter
    cache = str(tmp_path / "tune.txt")
    best, table = b.autotune(calib_sweeps=32, cache_path=cache)
    assert len(table) >= 12
    assert best in [t for t, _ in table]
    assert all(rate > 0 for _, rate in table)
    assert b.get_tuning() == best
    _same(_state(b), before)
    assert b.sweep_counter == t_before
    text = open(cache).read().split()
    assert len(text) == 7 and [int(x) for x in text[1:]] == [best[k] for k in nfm.TUNING_FIELDS]
    best2, table2 = b.autotune(calib_sweeps=32, cache_path=cache)    # cached: no measurement
    assert best2 == best and table2 == []
    b.run_sweeps(20)
    after = _state(b)
    c = _batch(nfm, orc, MIX, 0)
    c.run_sweeps(10)
    c.run_sweeps(20)
    _same(_state(c), after)
    b.close()
    c.close()


def test_small_lattice_queue_and_split_fallback(nfm, orc):
    """Batches of sizes up to 8 and up to 10 run the queue forms compiled for them; schedule 2 on a
    batch of one size falls back to the plain queue; all bit for bit as the per-size launches."""
    n = 30
    for Ls in ([4, 8, 6, 8, 4, 2], [8, 8, 8], [10, 4, 8, 10, 6]):
        ref = _batch(nfm, orc, Ls, n)
        ref.set_tuning(schedule=0)
        ref.run_sweeps(n)
        want = _state(ref)
        ref.close()
        for sch in (1, 2):
            b = _batch(nfm, orc, Ls, n)
            b.set_tuning(schedule=sch, sweeps_per_launch=8)
            b.run_sweeps(n)
            _same(_state(b), want)
            b.close()


def test_split_with_more_large_waves_than_its_share(nfm, orc):
    """More waves of the largest size than half the SIMDs: the SIMD-exclusive part is a
    persistent queue over more items than workgroups; bit for bit as the per-size launches."""
    import torch
    n_simd = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    Ls = [12] * (n_simd // 2 + 9) + [4, 6, 4]
    n = 3
    print("split: largest size", Ls.count(12), "waves for", n_simd // 2, "SIMDs", flush=True)
    ref = _batch(nfm, orc, Ls, n)
    ref.set_tuning(schedule=0)
    ref.run_sweeps(n)
    want = _state(ref)
    ref.close()
    b = _batch(nfm, orc, Ls, n)
    b.set_tuning(schedule=2, sweeps_per_launch=2)
    b.run_sweeps(n)
    assert b.last_kernel() == "k_sweeps_queue_solo"
    _same(_state(b), want)
    b.close()
