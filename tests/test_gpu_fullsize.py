"""GPU parity at the benchmark's full workload sizes, in the launch configuration it times.

The batches are set up exactly as the benchmark sets them up (its own set-up routine and launch
settings): L = 6 x 1024 realizations and L = 8 x 4096 under the weight recursion (power-law
targets, launches of 1000 sweeps, one weight update between two rounds), tempering at
L = 8 x 4096 with two sets of 32 temperatures per realization, and the mixed batch
L = 4/6/8/10/12 x 4096/2048/1024/512/256 under the persistent queue. Walkers of different
realizations never interact and within a round the table is fixed, so one realization's run
depends on nothing but its id: the oracle replays a sample of realizations (the first, the last
and some in between) on their own, and their spins, walker records, histograms, realization sums,
tempering slots and exchange counters are compared bit for bit, the weight update to 1e-12.
Properties that hold at any size are checked over the whole batch: every walker adds one count
per sweep to its realization's histogram, the realization sums are the sums of their walkers,
and every tempering set holds each temperature exactly once.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_08560_amd import nfm as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def bench():
    import bench as bm
    return bm


FIELDS = ("E", "E_min", "rt_state", "new_min", "rt_count", "t_first", "t_last")


def _parallel(fn, items):
    """The oracle's replays of independent realizations side by side (its C routines hold no
    shared state and ctypes releases the interpreter lock while they run)."""
    items = list(items)
    with ThreadPoolExecutor(max_workers=max(1, min(16, len(items)))) as pool:
        return list(pool.map(fn, items))


def _sample_ids(n, k, seed):
    rng = np.random.default_rng(seed)
    inner = rng.choice(np.arange(1, n - 1), size=k, replace=False) if n > 2 else []
    return sorted({0, n - 1, *(int(x) for x in inner)})


def _tables_agree(thr, ref):
    """Device-built thresholds against the oracle's: equal but where exp's last bit decides
    floor(x 2^32) (then by one)."""
    assert thr.shape == ref.shape
    diff = np.argwhere(thr != ref)
    assert len(diff) <= 3, len(diff)
    for r, u in diff:
        assert abs(int(thr[r, u]) - int(ref[r, u])) == 1


def _normwise(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _oracle_tables(orc, rz, st, profile):
    S, lnP, lnW = orc.rec_weights(rz.K, rz.eb, st.k_lo, st.k_top, *profile, st.b)
    thr, row0 = orc.build_thresholds(rz.K, lnW[st.k_lo:st.k_top + 1], st.k_lo, st.k_top)
    return thr, row0, lnW, lnP


def _sync_tables(b, orc, refs, profile):
    """Oracle tables of the sampled realizations for the coming round; where the device's table
    differs in exp's last bit the device takes the oracle's, so that both run the same chain."""
    tabs = {}
    for r, (rz, st) in refs.items():
        thr, row0, lnW, lnP = _oracle_tables(orc, rz, st, profile)
        dthr, drow0 = b.get_thresholds(r)
        assert drow0 == row0, r
        _tables_agree(dthr, thr)
        if not np.array_equal(dthr, thr):
            b.set_thresholds(r, thr, row0)
        tabs[r] = (thr, row0, lnW, lnP)
    return tabs


def _compare_round(b, orc, refs, tabs, n_sweeps, W):
    """Device state after a round against the oracle's replay of the sampled realizations."""
    ws = b.read_walkers()
    H = b.read_histograms()
    st_dev = b.read_realizations()
    def replay(r):
        rz, st = refs[r]
        thr, row0, _, _ = tabs[r]
        return orc.sample(rz, thr, row0, rz.eb + 4 * st.k_lo, 0, n_sweeps)[0]
    hists = dict(zip(refs, _parallel(replay, refs)))
    for r, (rz, st) in refs.items():
        Hr = hists[r]
        w0 = b.walker_offset(r)
        got = b.get_spins(w0, W).reshape(W, rz.N)
        assert np.array_equal(got, rz.S), (r, "spins")
        for f in FIELDS:
            assert np.array_equal(ws[f][w0:w0 + W], rz.w[f]), (r, f)
        off = b.level_offset(r)
        assert np.array_equal(H[off:off + rz.K], Hr), (r, "histogram")
    # at any size: one count per walker and sweep, realization sums are their walkers' sums
    for r in range(b.n_real):
        off, w0 = b.level_offset(r), b.walker_offset(r)
        K = b.levels(r)
        assert int(H[off:off + K].sum()) == W * n_sweeps, r
    _check_sums(ws, st_dev, b, W)
    return hists


def _check_sums(ws, st, b, W):
    n = b.n_real
    rt = ws["rt_count"].reshape(n, W)
    tf = ws["t_first"].reshape(n, W).astype(np.int64)
    tl = ws["t_last"].reshape(n, W).astype(np.int64)
    has = rt > 0
    assert np.array_equal(st["rt_count"], rt.sum(axis=1))
    assert np.array_equal(st["rt_time"], np.where(has, tl - tf, 0).sum(axis=1))
    assert np.array_equal(st["E_min"], ws["E_min"].reshape(n, W).min(axis=1))
    assert np.array_equal(st["walkers_with_trips"], has.sum(axis=1))
    assert np.all(ws["E_min"] <= ws["E"])


def _update_and_compare(b, orc, refs, tabs, hists):
    info = b.rec_update(0.5)
    for r, (rz, st) in refs.items():
        _, _, lnW, lnP = tabs[r]
        k_min = (int(rz.w["E_min"].min()) - rz.eb) // 4
        st.k_lo, flat = orc.rec_update(rz.K, st.k_lo, st.k_top, min(k_min, st.k_lo), lnW, lnP, hists[r],
                                       st.b, st.p, st.visited)
        assert info["k_lo"][r] == st.k_lo, r
        assert abs(info["flatness"][r] - flat) <= 1e-12 * max(flat, 1e-300), r
        d = b.rec_get_state(r)
        sl = slice(st.k_lo, st.k_top + 1)
        assert _normwise(d["b"][sl], st.b[sl]) <= 1e-12, r
        assert _normwise(d["p"][sl], st.p[sl]) <= 1e-12, r


def _refs(orc, bench, Ls, ids, W):
    out = {}
    for r in ids:
        rz = orc.make_realization(Ls[r], bench.DSEED, r, bench.DSEED + 1, W)
        out[r] = (rz, orc.recursion_init(rz))
    return out


@pytest.mark.parametrize("config,form,n_sample", [("c2", "k_sweeps_ws<6>", 6), ("c3", "k_sweeps<8>", 4)])
def test_recursion_full_size(nfm, orc, bench, config, form, n_sample):
    """Two rounds of the benchmark's step (sweeps in launches of 1000, the device weight update)
    at the full size, the sampled realizations replayed by the oracle."""
    mix, W, _, _ = bench.CONFIGS[config]
    profile = bench.PROFILES[config]
    print("full size:", config, mix, "walkers", W, flush=True)
    b, Ls = bench.setup(nfm, mix, W, profile)
    b.set_tuning(speculate=-1, sweeps_per_launch=1000, ws=0)       # as the benchmark times it
    ids = _sample_ids(len(Ls), n_sample, 1)
    refs = _refs(orc, bench, Ls, ids, W)
    tabs = _sync_tables(b, orc, refs, profile)
    b.run_sweeps(2000)
    assert b.last_kernel() == form
    hists = _compare_round(b, orc, refs, tabs, 2000, W)
    _update_and_compare(b, orc, refs, tabs, hists)
    print("full size:", config, "second weight round", flush=True)
    tabs = _sync_tables(b, orc, refs, profile)
    b.run_sweeps(1000)
    _compare_round(b, orc, refs, tabs, 1000, W)
    b.close()


def test_mixed_queue_full_size(nfm, orc, bench):
    """The mixed batch under the persistent queue and the split launch (launches of 256
    sweeps, with and without speculation: the forms the autotuner picks from), two realizations
    of every size against the oracle; all forms agree on the whole batch bit for bit."""
    mix, W, _, _ = bench.CONFIGS["c4"]
    profile = bench.PROFILES["c4"]
    Ls = [L for L, R in mix for _ in range(R)]
    ids, start = [], 0
    for L, R in mix:
        ids += [start, start + R - 1]
        start += R
    refs = None
    results = []
    for schedule, spec in ((1, 0), (1, 1), (2, 0), (2, 1)):
        print("full size: c4, schedule", schedule, "speculate", spec, flush=True)
        b, _ = bench.setup(nfm, mix, W, profile)
        b.set_tuning(speculate=spec, sweeps_per_launch=256, schedule=schedule)
        if refs is None:
            refs = _refs(orc, bench, Ls, ids, W)
            tabs = _sync_tables(b, orc, refs, profile)
            ref_tabs = tabs
        else:
            for r, (thr, row0, _, _) in ref_tabs.items():
                dthr, drow0 = b.get_thresholds(r)
                if not np.array_equal(dthr, thr):
                    b.set_thresholds(r, thr, row0)
        b.run_sweeps(512)
        form = ("k_sweeps_queue_spec" if spec else "k_sweeps_queue") + ("_solo" if schedule == 2 else "")
        assert b.last_kernel() == form
        if not results:
            _compare_round(b, orc, refs, ref_tabs, 512, W)
        ws = b.read_walkers()
        results.append((ws, b.read_histograms(), b.get_spins(0, b.n_walkers)))
        b.close()
    # every form agrees on the whole batch, bit for bit
    (w0, h0, s0) = results[0]
    for (w1, h1, s1) in results[1:]:
        for f in FIELDS:
            assert np.array_equal(w0[f], w1[f]), f
        assert np.array_equal(h0, h1)
        assert np.array_equal(s0, s1)


def test_tempering_full_size(nfm, orc, bench):
    """Tempering at the full size (L = 8 x 4096, two sets of 32 temperatures per realization,
    exchanges every sweep, launches of 1000 sweeps)."""
    mix, W, _, _ = bench.CONFIGS["c3pt"]
    M = 32
    print("full size: c3pt", mix, flush=True)
    b, Ls = bench.setup(nfm, mix, W, None)
    b.set_tuning(speculate=-1, sweeps_per_launch=1000)
    n = 2000
    b.pt_run_sweeps(n)
    assert b.last_kernel() == "k_sweeps_pt<8>"
    T = np.array([0.2 * 10.0 ** (m / (M - 1)) for m in range(M)])
    ws = b.read_walkers()
    slots = b.pt_slots()
    acc = b.pt_exchanges(M)
    sets_r = (W // 64) * (64 // M)
    ids = _sample_ids(len(Ls), 3, 2)
    L = mix[0][0]
    N = L ** 3
    e_bot, e_top = int(-1.66 * N), int(-1.40 * N)
    metro, swap = orc.pt_metro_table(T), orc.pt_swap_table(T, 3 * N // 2 + 1)

    def replay(rg):
        ps = orc.make_pt_set(L, bench.DSEED, rg[0], bench.DSEED + 1, M, set_index=rg[1])
        a_ref = np.zeros(M - 1, np.uint64)
        orc.pt_sweeps(ps, metro, swap, e_bot, e_top, n, swap_acc=a_ref)
        return ps, a_ref
    keys = [(r, g) for r in ids for g in range(sets_r)]
    ref = dict(zip(keys, _parallel(replay, keys)))
    for r in ids:
        assert Ls[r] == L
        dm, dsw = b.pt_tables(r)
        assert np.array_equal(dm, metro) and np.array_equal(dsw, swap), r
        w0 = b.walker_offset(r)
        S_dev = b.get_spins(w0, W).reshape(W, N)
        for g in range(sets_r):
            ps, a_ref = ref[(r, g)]
            k0 = ps.walker0
            sl = slice(w0 + k0, w0 + k0 + M)
            assert np.array_equal(S_dev[k0:k0 + M], ps.S), (r, g, "spins")
            for f in FIELDS:
                assert np.array_equal(ws[f][sl], ps.w[f]), (r, g, f)
            assert np.array_equal(slots[sl], ps.slot), (r, g, "slots")
            assert np.array_equal(acc[r * sets_r + g], a_ref), (r, g, "exchanges")
    # at any size: every set holds each temperature slot exactly once
    per = slots.reshape(-1, 64)[:, :(64 // M) * M].reshape(-1, M)
    assert np.array_equal(np.sort(per, axis=1), np.broadcast_to(np.arange(M), per.shape))
    _check_sums(ws, b.read_realizations(), b, W)
    b.close()
