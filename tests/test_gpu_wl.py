"""GPU parity of the batched Wang-Landau estimate against the oracle.

Each step: the device's histogram of the step (its sampling is checked against the oracle on the
first step, from the initial state with the device's table), then ln g, the stage histogram, ln f,
stage, flatness and done flag after the device update against the oracle's update of the same
histogram (FP64, bit for bit: ln f is a power of two and the histogram integer), and the device's
table against the oracle's thresholds of the same weights (within one unit where exp's last bit
decides). Finally the hand-over to the recursion: k_lo and the steps b.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DSEED, WSEED = 20110856, 0x2468ACE


@pytest.fixture(scope="module")
def nfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_08560_amd import nfm as m
    m.lib()
    return m


def test_wl_matches_oracle(nfm, orc):
    Ls, W, first = [4, 4, 6], 64, 60
    b = nfm.Batch(Ls, [W] * 3, DSEED, WSEED, first_real_id=first)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    b.wl_init(1.0)
    refs = []
    for r, L in enumerate(Ls):
        J = orc.couplings(L, DSEED, first + r)
        refs.append(orc.wl_init(orc.n_levels(L, J), orc.e_base(L, J), 1.0))
    # the first step's sampling from the initial state, with the device's table
    rz = orc.make_realization(4, DSEED, first, WSEED, W)
    thr, row0 = b.get_thresholds(0)
    H0, _ = orc.sample(rz, thr, row0, -10 ** 6, 10 ** 6, 30)
    # with ln f = 1 the stage histogram of L = 4 first reaches min/mean >= 0.35 at step 12
    for step in range(18):
        b.run_sweeps(30 if step == 0 else 40)
        H = b.read_histograms()
        if step == 0:
            assert np.array_equal(H[:len(H0)], H0)
        info = b.wl_update(flat_tol=0.35, ln_f_final=0.05)
        for r, L in enumerate(Ls):
            off = b.level_offset(r)
            st = refs[r]
            orc.wl_update(st, H[off:off + len(st.lng)], 0.35, 0.05)
            lng, hst, inf = b.wl_get(r)
            n = len(st.lng)
            assert np.array_equal(lng[:n], st.lng), (step, r)
            assert np.array_equal(hst[:n], st.hst), (step, r)
            assert inf["ln_f"] == st.ln_f and inf["stage"] == st.stage and bool(inf["done"]) == st.done
            assert inf["flatness"] == st.flatness and inf["updates"] == st.updates
            assert info[r]["ln_f"] == st.ln_f
            if not st.done:
                thr_d, row0_d = b.get_thresholds(r)
                thr_o, row0_o = orc.wl_thresholds(st, n)
                assert row0_d == row0_o and thr_d.shape == thr_o.shape
                assert np.abs(thr_d.astype(np.int64) - thr_o.astype(np.int64)).max() <= 1
    assert any(st.stage > 0 for st in refs)
    b.wl_to_rec()
    for r, L in enumerate(Ls):
        k_lo, steps = orc.wl_to_rec_steps(refs[r])
        rs = b.rec_get_state(r)
        assert int(rs["info"]["k_lo"]) == k_lo and int(rs["info"]["k_top"]) == refs[r].k_top
        assert np.array_equal(rs["b"][:len(steps)], steps)
        assert np.array_equal(rs["visited"][:len(steps)] != 0, refs[r].lng > 0)
    b.close()
