"""Pins for the oracle's weight-seeding parts: frustration statistics, histogram bins,
the grid-to-steps conversion, the seeded recursion, and the fp64 network.

Independent facts used:
  * closed forms: every statistic of the ferromagnet (all J = +1), and of the ferromagnet
    with one negative bond (which frustrates the four plaquettes and the four cubes that
    hold it, and lowers two site sums by 2);
  * gauge invariance: J_ij -> e_i J_ij e_j with e = +-1 changes bonds but no plaquette or
    cube product, so every frustration statistic is unchanged;
  * cubes always have an even number of frustrated faces (fractions sum to 1);
  * a linear curve S(E)/N = a E/N gives DOS steps b = 4a on every level; a decreasing curve
    or a non-finite value is rejected; where a curve turns down its steps are flat;
  * with the exact DOS of an L = 3 realization as the seed, the first sampling round is
    already flat over the whole range, so the seeded iteration converges at once while the
    plain start needs several rounds;
  * the network's gradient equals central finite differences of its loss; Adam's first
    step is -lr g / (|g| + eps) elementwise; GELU(1) = Phi(1) = 0.8413447460685429.
"""
import math

import numpy as np
import pytest


def _ferro(L):
    return np.ones(3 * L ** 3, np.int8)


def test_features_ferromagnet_and_one_bond(orc):
    L = 4
    N = L ** 3
    f = orc.features(L, _ferro(L))
    want = np.zeros(16)
    want[9] = 1.0      # every cube has 0 frustrated faces
    want[13] = 1.0     # site sums all 6: mean/6 = 1, no spread
    assert np.allclose(f, want, atol=0, rtol=0)
    J = _ferro(L)
    i0 = 1 + L * 2 + L * L * 3
    J[1 * N + i0] = -1   # one y bond
    f = orc.features(L, J)
    assert f[0] == 2 / N and f[1] == 2 / N and f[2] == 0.0          # (x,y) and (y,z) hold the y bond
    assert f[3] == 4 / (3 * N)
    assert f[4] == 0 and f[5] == 1 / N and f[6] == 0 and f[7] == 1 / (3 * N)
    assert f[8] == 1.0
    assert f[9] == (N - 4) / N and f[10] == 4 / N and f[11] == 0 and f[12] == 0
    sums = np.full(N, 6.0)
    sums[:2] = 4.0
    mean = sums.mean()
    assert abs(f[13] - mean / 6) < 1e-15
    assert abs(f[14] - ((sums - mean) ** 2).mean() / 6) < 1e-15
    assert abs(f[15] - ((sums - mean) ** 4).mean() / 96) < 1e-15


@pytest.mark.parametrize("L", [3, 4, 5])
def test_features_gauge_invariant(orc, L):
    N = L ** 3
    rng = np.random.default_rng(L)
    J = orc.couplings(L, 99, L)
    f = orc.features(L, J)
    assert abs(f[9:13].sum() - 1.0) < 1e-15
    eps = rng.choice(np.array([-1, 1], np.int8), N)
    Jg = J.copy()
    for d in range(3):
        for i in range(N):
            x, y, z = i % L, (i // L) % L, i // (L * L)
            j = [((x + 1) % L) + L * y + L * L * z, x + L * ((y + 1) % L) + L * L * z,
                 x + L * y + L * L * ((z + 1) % L)][d]
            Jg[d * N + i] = J[d * N + i] * eps[i] * eps[j]
    g = orc.features(L, Jg)
    for k in (0, 1, 2, 3, 9, 10, 11, 12):
        assert g[k] == f[k], k


def test_hist_bins_by_hand(orc):
    N, eb = 64, -192
    K = 97
    H = np.zeros(K, np.uint64)
    # E = -192 (E/N = -3, clipped to bin 0), -100 (-1.5625 -> bin 14), -2 (-0.03125 -> bin 63), +8 (clipped 63)
    for E, c in ((-192, 3), (-100, 5), (-2, 0), (8, 2)):
        H[(E - eb) // 4] = c
    H[(-4 - eb) // 4] = 10   # E/N = -0.0625 -> bin 62
    out = orc.hist_bins(K, eb, N, H)
    tot = 20.0
    assert out[0] == 3 / tot and out[14] == 5 / tot and out[62] == 10 / tot and out[63] == 2 / tot
    assert abs(out.sum() - 1.0) < 1e-15


def test_seed_from_linear_curve_and_rejection(orc):
    N, eb = 216, -648
    k_top = -eb // 4
    a = 0.7
    e = -2.0 + 2.0 * np.arange(256) / 255.0
    y = (a * e).astype(np.float32)
    b = np.zeros(k_top + 10)
    k_s = orc.seed_from_grid(N, eb, k_top, y, b)
    assert k_s == (-2 * N - eb + 3) // 4
    assert np.allclose(b[k_s:k_top - 1], 4 * a, atol=N * 2e-6)   # float32 curve: N x (a few ulp)
    assert (b[:k_s] == 0).all() and (b[k_top:] == 0).all()
    b2 = np.zeros_like(b)
    assert orc.seed_from_grid(N, eb, k_top, -y, b2) == -1            # decreasing: no information
    assert not b2.any()
    y_nan = y.copy()
    y_nan[100] = np.nan
    assert orc.seed_from_grid(N, eb, k_top, y_nan, b2) == -1
    # increasing above e = -1.5, decreasing below: flat steps below the turn
    y3 = np.where(e >= -1.5, a * e, a * (-3.0 - e)).astype(np.float32)
    b3 = np.zeros_like(b)
    assert orc.seed_from_grid(N, eb, k_top, y3, b3) == k_s
    E = eb + 4 * np.arange(len(b3))
    assert (b3[(E >= -1.5 * N + 8) & (E < 4 * k_top + eb)] > 0).all()
    assert not b3[(E < -1.5 * N - 8)].any()


def test_seeded_iteration_with_exact_dos_converges_at_once(orc):
    L, W, n_sw = 3, 32, 400
    for rid in (2, 5):
        rz_plain = orc.make_realization(L, 4242, rid, 77, W)
        rz_seed = orc.make_realization(L, 4242, rid, 77, W)
        g = orc.brute_dos(L, rz_plain.J).astype(np.float64)
        K, eb = rz_plain.K, rz_plain.eb
        k_top = rz_plain.k_top
        lng = np.full(K, -np.inf)
        lng[g > 0] = np.log(g[g > 0])
        k_g = int(np.argmax(g > 0))
        st_p = orc.recursion_init(rz_plain)
        st_s = orc.recursion_init(rz_seed)
        st_s.b[k_g:k_top] = lng[k_g + 1:k_top + 1] - lng[k_g:k_top]
        log_s = orc.weight_iterations(rz_seed, st_s, 12, n_sw, f_tol=0.5, k_seed=k_g)
        log_p = orc.weight_iterations(rz_plain, st_p, 12, n_sw, f_tol=0.5)
        assert log_s[0][2] > 0.5, log_s
        assert len(log_s) <= 2 and log_s[-1][3], log_s
        assert len(log_p) >= 3, log_p


def test_rec_ext_reduces_to_plain(orc):
    rng = np.random.default_rng(3)
    K, eb, k_lo, k_top = 60, -120, 12, 30
    b = np.zeros(K)
    b[5:k_top] = rng.uniform(0.5, 2.0, k_top - 5)
    for prof, dE, al in ((0, 1.0, 0.0), (1, 1.0, -1.0), (2, 1.0, 0.0)):
        S0, P0, W0 = orc.rec_weights(K, eb, k_lo, k_top, prof, dE, al, b)
        S1, P1, W1 = orc.rec_weights_ext(K, eb, k_lo, k_top, k_lo, prof, dE, al, b)
        assert np.array_equal(S0, S1) and np.array_equal(W0, W1) and np.array_equal(P0, P1)
        S2, P2, W2 = orc.rec_weights_ext(K, eb, k_lo, k_top, 5, prof, dE, al, b)
        assert np.array_equal(W2[k_lo:], W0[k_lo:])
        # below k_lo: S continues with the seeded steps, the profile is frozen
        assert np.allclose(S2[5:k_lo], S0[k_lo] - np.cumsum(b[5:k_lo][::-1])[::-1], atol=1e-12)
        assert (P2[5:k_lo] == P0[k_lo]).all()
    H = rng.integers(0, 50, K).astype(np.uint64)
    lnW = rng.normal(0, 1, K)
    lnP = np.zeros(K)
    for seeded in (0, 1):
        b1, p1, v1 = b.copy(), np.zeros(K), np.zeros(K, np.uint8)
        b2, p2, v2 = b.copy(), np.zeros(K), np.zeros(K, np.uint8)
        r1 = orc.rec_update(K, k_lo, k_top, 8, lnW, lnP, H, b1, p1, v1)
        r2 = orc.rec_update_ext(K, k_lo, k_top, k_lo, seeded, 8, lnW, lnP, H, b2, p2, v2)
        if not seeded:
            assert r1 == r2 and np.array_equal(b1, b2)
        else:
            # seeded: levels 8..11 keep their own steps before the update pass
            assert r1[0] == r2[0]
            assert not np.array_equal(b1[8:k_lo], b2[8:k_lo])


def test_mlp_gradient_matches_finite_differences():
    from oracle import mlp
    rng = np.random.default_rng(0)
    theta = mlp.init_params(1)
    theta[mlp.N_PARAM - 256:] = rng.normal(0, 0.1, 256)   # nonzero output biases
    norm = np.stack([rng.normal(0, 1, mlp.D_IN), rng.uniform(0.5, 2.0, mlp.D_IN)])
    B = 5
    X = rng.normal(0, 1, (B, mlp.D_IN))
    T = rng.normal(0, 1, (B, mlp.D_OUT))
    M = (rng.random((B, mlp.D_OUT)) < 0.7).astype(np.float64)
    L, g = mlp.loss_and_grad(theta, norm, X, T, M)
    assert abs(L - mlp.loss(theta, norm, X, T, M)) < 1e-15
    P = mlp.unflatten(np.arange(mlp.N_PARAM, dtype=np.float64))
    idx = []
    for name in ("W0", "b0", "W1", "b1", "W2", "b2", "W3", "b3"):
        flat = P[name].reshape(-1).astype(int)
        idx += list(rng.choice(flat, 6, replace=False))
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, norm, X, T, M) - mlp.loss(tm, norm, X, T, M)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    # padding rows of W0 see zero inputs: zero gradient
    Pg = mlp.unflatten(g)
    assert not Pg["W0"][mlp.D_IN:].any()


def test_adam_first_step_and_gelu_value():
    from oracle import mlp
    assert abs(mlp.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert mlp.gelu(np.array(0.0)) == 0.0
    rng = np.random.default_rng(5)
    theta = rng.normal(0, 1, 50)
    g = rng.normal(0, 1, 50)
    m, v = np.zeros(50), np.zeros(50)
    t0 = theta.copy()
    mlp.adam_step(theta, g, m, v, 1, 1e-3)
    assert np.allclose(theta - t0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)


def test_rec_targets_linear_estimate(orc):
    """S linear in E (S = c (E - E_top)) gives y = c (e N - E_top)/N on the defined grid points,
    masked below E(k_lo)."""
    N, eb = 216, -648
    K = 3 * N // 2 + 1
    k_lo, k_top = 60, 162
    c = 0.35
    E = eb + 4 * np.arange(K)
    S = np.zeros(K)
    S[k_lo:k_top + 1] = c * (E[k_lo:k_top + 1] - E[k_top])
    y, m = orc.rec_targets(N, eb, k_lo, k_top, S)
    e = -2.0 + 2.0 * np.arange(256) / 255.0
    inside = e * N >= eb + 4 * k_lo
    assert np.array_equal(m, inside.astype(float))
    assert np.allclose(y[inside], c * (e[inside] * N - E[k_top]) / N, atol=1e-12)
    assert not y[~inside].any()
