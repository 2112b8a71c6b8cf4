"""GPU parity: libnfm (HIP, gfx950) against the CPU oracle, element by element.

Integer work is compared bit for bit: couplings, initial spins, energies, spin
configurations after sweeps, energy traces, histograms, minima and round-trip
counters. Thresholds built on the device from FP64 log-weights may differ from the
oracle's only where floor(x 2^32) sits within exp's rounding of an integer.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DSEED, WSEED = 20110856, 0x5EED1234ABCD


@pytest.fixture(scope="module")
def nfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_08560_amd import nfm as m
    m.lib()
    return m


def _oracle_walkers(orc, L, rid, W, seed=WSEED):
    J = orc.couplings(L, DSEED, rid)
    S = [orc.spins(L, seed, rid, w) for w in range(W)]
    return J, S


@pytest.mark.parametrize("L", [2, 4, 6, 8, 10, 12])
def test_couplings_spins_energies(nfm, orc, L):
    n_real, W = 3, 64
    b = nfm.Batch([L] * n_real, [W] * n_real, DSEED, WSEED, first_real_id=11)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    words = b.get_couplings(0, n_real).reshape(n_real, -1)
    ws = b.read_walkers()
    for r in range(n_real):
        J, S = _oracle_walkers(orc, L, 11 + r, W)
        assert np.array_equal(words[r], nfm.pack_couplings(J, L))
        assert b.levels(r) == orc.n_levels(L, J)
        assert b.e_base(r) == orc.e_base(L, J)
        got = b.get_spins(b.walker_offset(r), W).reshape(W, L ** 3)
        for w in range(W):
            assert np.array_equal(got[w], S[w]), (r, w)
            E = orc.energy(L, J, S[w])
            assert ws["E"][r * W + w] == E and ws["E_min"][r * W + w] == E
    b.close()


def test_set_get_roundtrip(nfm, orc):
    L, W = 6, 128
    b = nfm.Batch([L, L], [W, W], DSEED, WSEED)
    rng = np.random.default_rng(4)
    J = [orc.couplings(L, 99, r) for r in range(2)]
    b.set_couplings(0, np.concatenate([nfm.pack_couplings(j, L) for j in J]))
    S = rng.choice(np.array([-1, 1], np.int8), size=(2 * W, L ** 3))
    b.set_spins(0, S)
    assert np.array_equal(b.get_spins(0, 2 * W).reshape(2 * W, -1), S)
    b.compute_energies()
    ws = b.read_walkers()
    for w in range(2 * W):
        assert ws["E"][w] == orc.energy(L, J[w // W], S[w])
    b.close()


def _weights(orc, L, J, beta, noise, seed):
    """Canonical-like log-weights with noise on a compact range, plus round-trip bounds
    near the equilibrium energy so that crossings happen within a few sweeps."""
    K, eb = orc.n_levels(L, J), orc.e_base(L, J)
    rng = np.random.default_rng(seed)
    E = eb + 4 * np.arange(K)
    lnw = -beta * E + np.cumsum(rng.normal(0.0, noise, K))
    k_top = (-eb + 3) // 4
    k_lo = max(0, (int(-1.2 * L ** 3) - eb) // 4)
    return K, eb, lnw, k_lo, k_top


# plain and speculative forms, each without (ws=1: expanded table / compact table) and with (ws=2,
# expanded table) the generator wave
@pytest.mark.parametrize("spec,ws", [(0, 1), (0, 2), (1, 1), (1, 2)])
@pytest.mark.parametrize("L,T", [(2, 40), (4, 32), (6, 24), (8, 16), (10, 10), (12, 8)])
def test_sweeps_bit_exact(nfm, orc, L, T, spec, ws):
    n_real, W, rid0 = 2, 64, 3
    print("sweeps bit-exact: L", L, "sweeps", T, "speculate", spec, "ws", ws, flush=True)
    b = nfm.Batch([L] * n_real, [W] * n_real, DSEED, WSEED, first_real_id=rid0, trace_capacity=T)
    b.set_tuning(speculate=spec, sweeps_per_launch=5, ws=ws)   # several launches per run: resume inside
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    refs = []
    for r in range(n_real):
        J, S = _oracle_walkers(orc, L, rid0 + r, W)
        K, eb, lnw, k_lo, k_top = _weights(orc, L, J, 0.35, 0.3, r)
        thr, row0 = orc.build_thresholds(K, lnw[k_lo:k_top + 1], k_lo, k_top)
        # bounds around the energies the walkers reach, picked from one oracle walker
        s0 = S[0].copy()
        w0 = orc.new_walkers(1, orc.energy(L, J, s0))
        tr = np.zeros(T, np.int32)
        orc.muca_sweeps(L, J, s0, w0, thr, row0, -10 ** 6, 10 ** 6, WSEED, rid0 + r, 0, 0, T, trace=tr)
        mid = int(np.median(tr[T // 2:]))
        e_bot, e_top = mid - 8, mid + 8
        b.set_thresholds(r, thr, row0)
        b.set_rt_bounds(r, e_bot, e_top)
        refs.append((J, S, K, thr, row0, e_bot, e_top))
    # two launches: resuming must not change anything
    b.run_sweeps(T // 2)
    b.run_sweeps(T - T // 2)
    form = {(0, 1): "k_sweeps_xt", (0, 2): "k_sweeps_ws", (1, 1): "k_sweeps_spec", (1, 2): "k_sweeps_ws_spec"}
    assert b.last_kernel() == f"{form[(spec, ws)]}<{L}>"   # the form under test is the one that ran
    ws = b.read_walkers()
    H = b.read_histograms()
    trace = b.read_trace()
    assert trace.shape == (n_real * W, T)
    spins = b.get_spins(0, n_real * W).reshape(n_real * W, L ** 3)
    trips = 0
    for r, (J, S, K, thr, row0, e_bot, e_top) in enumerate(refs):
        Href = np.zeros(K, np.uint64)
        for w in range(W):
            g = r * W + w
            s = S[w].copy()
            wr = orc.new_walkers(1, orc.energy(L, J, s))
            tr = np.zeros(T, np.int32)
            orc.muca_sweeps(L, J, s, wr, thr, row0, e_bot, e_top, WSEED, rid0 + r, w, 0, T, hist=Href, trace=tr)
            assert np.array_equal(spins[g], s), (r, w)
            assert np.array_equal(trace[g], tr), (r, w)
            for f in ("E", "E_min", "rt_state", "new_min", "rt_count", "t_first", "t_last"):
                assert ws[f][g] == wr[f][0], (f, r, w, ws[g], wr[0])
            trips += int(wr["rt_count"][0])
        off = b.level_offset(r)
        assert np.array_equal(H[off:off + K], Href), r
    st = b.read_realizations()
    for r in range(n_real):
        sl = ws[r * W:(r + 1) * W]
        has = sl["rt_count"] > 0
        assert st["rt_count"][r] == sl["rt_count"].sum()
        assert st["rt_time"][r] == (sl["t_last"][has] - sl["t_first"][has]).sum()
        assert st["E_min"][r] == sl["E_min"].min()
        assert st["new_min"][r] == int(sl["new_min"].max())
        assert st["walkers_with_trips"][r] == int(has.sum())
    if L >= 4:
        assert trips > 0, "bounds chosen so that round trips complete"
    b.close()


def test_mixed_sizes_one_batch(nfm, orc):
    """Realizations of different L in one batch; a few walkers of each checked."""
    Ls, Ws, T = [4, 8, 6, 12, 10, 8], [64, 128, 64, 64, 64, 64], 6
    b = nfm.Batch(Ls, Ws, DSEED, WSEED, first_real_id=100)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    refs = []
    for r, L in enumerate(Ls):
        J = orc.couplings(L, DSEED, 100 + r)
        K, eb, lnw, k_lo, k_top = _weights(orc, L, J, 0.3, 0.2, 7 + r)
        thr, row0 = orc.build_thresholds(K, lnw[k_lo:k_top + 1], k_lo, k_top)
        b.set_thresholds(r, thr, row0)
        b.set_rt_bounds(r, int(-1.1 * L ** 3), int(-0.9 * L ** 3))
        refs.append((J, thr, row0))
    b.run_sweeps(T)
    ws = b.read_walkers()
    for r, L in enumerate(Ls):
        J, thr, row0 = refs[r]
        for w in (0, Ws[r] - 1, 37):
            g = b.walker_offset(r) + w
            s = orc.spins(L, WSEED, 100 + r, w)
            wr = orc.new_walkers(1, orc.energy(L, J, s))
            orc.muca_sweeps(L, J, s, wr, thr, row0, int(-1.1 * L ** 3), int(-0.9 * L ** 3), WSEED, 100 + r, w, 0, T)
            assert np.array_equal(b.get_spins(g, 1), s)
            for f in ("E", "E_min", "rt_state", "new_min", "rt_count", "t_first", "t_last"):
                assert ws[f][g] == wr[f][0], (f, r, w)
    b.close()


def _ratio(lnw, k_lo, k_top, k, m):
    """W(k+m)/W(k) with the documented continuation of the step log-weights."""
    def d(j):
        j = max(j, k_lo)
        return 0.0 if j >= k_top else lnw[j + 1] - lnw[j]
    s = 0.0
    if m > 0:
        for j in range(k, k + m):
            s += d(j)
        return math.exp(s)
    if m < 0:
        for j in range(k + m, k):
            s += d(j)
        return math.exp(-s)
    return 1.0


@pytest.mark.parametrize("L", [4, 8, 12])
def test_device_tables_match_oracle(nfm, orc, L):
    n_real = 3
    b = nfm.Batch([L] * n_real, [64] * n_real, DSEED, WSEED, first_real_id=40)
    b.init_couplings()
    lnw_all = np.zeros(b.levels_total)
    klo, ktop, expect = [], [], []
    rng = np.random.default_rng(L)
    for r in range(n_real):
        J = orc.couplings(L, DSEED, 40 + r)
        K, eb = orc.n_levels(L, J), orc.e_base(L, J)
        k_top = (-eb + 3) // 4
        k_lo = [0, 5, k_top - 2][r]
        lnw = np.cumsum(rng.normal(0.5, 2.0, K))
        lnw_all[b.level_offset(r):b.level_offset(r) + K] = lnw
        klo.append(k_lo)
        ktop.append(k_top)
        expect.append(orc.build_thresholds(K, lnw[k_lo:k_top + 1], k_lo, k_top) + (lnw, k_lo, k_top))
    b.set_weights_lnw(lnw_all, klo, ktop)
    for r in range(n_real):
        thr_ref, row0_ref, lnw, k_lo, k_top = expect[r]
        thr, row0 = b.get_thresholds(r)
        assert row0 == row0_ref and thr.shape == thr_ref.shape
        diff = np.argwhere(thr != thr_ref)
        for rr, u in diff:
            # the only allowed differences: exp's last bit decides floor(x 2^32)
            assert abs(int(thr[rr, u]) - int(thr_ref[rr, u])) == 1, (r, rr, u)
            y = math.ldexp(_ratio(lnw, k_lo, k_top, row0 + rr, 3 - u), 32)
            assert abs(y - round(y)) < 1e-5, (r, rr, u, y)
        assert len(diff) <= 2, (r, len(diff))
    b.close()


def test_invalid_arguments(nfm):
    b = nfm.Batch([4], [64], DSEED, WSEED)
    with pytest.raises(nfm.NfmError) as e:
        b.run_sweeps(1)   # couplings / tables missing
    assert e.value.status in (nfm.NFM_ESTATE,)
    b.init_couplings()
    with pytest.raises(nfm.NfmError) as e:
        b.set_thresholds(0, np.zeros((b.levels(0) + 1, 8), np.uint32), 0)
    assert e.value.status == nfm.NFM_EINVAL
    with pytest.raises(nfm.NfmError):
        b.set_rt_bounds(3, 0, 0)
    b.close()
