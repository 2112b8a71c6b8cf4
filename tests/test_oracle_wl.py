"""Pins of the Wang-Landau oracle (batched form).

* The update's arithmetic: after one step ln g = ln f0 H exactly, the stage histogram is H, and a
  flat stage halves ln f and clears it.
* Convergence to the exact density of states: for two realizations at L = 2 the estimate, run
  to a small ln f, matches ln g from complete enumeration up to the statistical error WL leaves at
  that ln f; the steps handed to the recursion sum to the estimate's differences.
"""
import numpy as np
import pytest

DSEED, WSEED = 20110856, 0x5151


def test_first_update_and_halving(orc):
    K, eb = 13, -24
    st = orc.wl_init(K, eb, 1.0)
    assert st.k_top == 6
    H = np.array([0, 3, 5, 4, 6, 2, 7, 9, 0, 0, 0, 0, 0], np.uint64)
    orc.wl_update(st, H, 0.9, 1e-3)
    assert np.array_equal(st.lng[:7], H[:7].astype(float)) and np.all(st.lng[7:] == 0)
    assert st.flatness == pytest.approx(2 / (27 / 6))
    assert st.stage == 0 and st.ln_f == 1.0
    orc.wl_update(st, np.array([0, 0, 0, 0, 0, 5, 0] + [0] * 6, np.uint64), 0.9, 1e-3)   # Hs = 3 5 4 6 7 7
    assert st.flatness == pytest.approx(3 / (32 / 6))
    flat = np.array([0, 9, 9, 9, 9, 9, 9] + [1] * 6, np.uint64)
    st2 = orc.wl_init(K, eb, 0.5)
    orc.wl_update(st2, flat, 0.9, 0.3)
    assert st2.stage == 1 and st2.ln_f == 0.25 and st2.done and not st2.hst.any()
    lng = st2.lng.copy()
    orc.wl_update(st2, flat, 0.9, 0.3)          # done: nothing moves
    assert np.array_equal(st2.lng, lng) and st2.updates == 1


@pytest.mark.parametrize("real_id", [0, 5])
def test_converges_to_exact_dos_at_L2(orc, real_id):
    L, W = 2, 8
    rz = orc.make_realization(L, DSEED, real_id, WSEED, W)
    K, eb = rz.K, orc.e_base(L, rz.J)
    g = orc.brute_dos(L, rz.J)
    st = orc.wl_init(K, eb, 1.0)
    for _ in range(4000):
        thr, row0 = orc.wl_thresholds(st, K)
        H, _ = orc.sample(rz, thr, row0, -10 ** 6, 10 ** 6, 20)
        orc.wl_update(st, H, 0.8, 2e-4)
        if st.done:
            break
    assert st.done
    ks = [k for k in range(st.k_top + 1) if g[k] > 0]
    assert all(st.lng[k] > 0 for k in ks)
    est = st.lng[ks] - st.lng[st.k_top]
    exact = np.log(g[ks].astype(float)) - np.log(float(g[st.k_top]))
    assert np.max(np.abs(est - exact)) < 0.15, (est, exact)
    k_lo, b = orc.wl_to_rec_steps(st)
    assert k_lo == ks[0]
    assert np.allclose(np.cumsum(b[k_lo:st.k_top])[-1], st.lng[st.k_top] - st.lng[k_lo])
