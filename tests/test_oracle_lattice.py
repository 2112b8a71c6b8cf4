"""Pins for the oracle's model (Eq. (1), Sec. II): energies, levels and the exact
density of states by enumeration.

Independent facts used:
  * closed forms: E(all up) = -sum J, E(staggered) = +sum J for even L;
  * the residue E = -3N + 2 n_minus (mod 4) of every reachable energy;
  * sum_E g(E) = 2^N, g even (global spin flip), g(E) = g(-E) for even L
    (gauge by (-1)^(x+y+z) on the bipartite lattice), g_J(E) = g_{-J}(-E);
  * the high-temperature series of ln Z, whose leading coefficients are sums of
    coupling products over the shortest closed loops of the periodic lattice;
  * a direct numpy enumeration of all 2^8 states at L = 2.
"""
import itertools
import math

import numpy as np
import pytest


def site(L, x, y, z):
    return (x % L) + L * (y % L) + L * L * (z % L)


def test_energy_closed_forms(orc):
    for L in (2, 3, 4, 6):
        N = L ** 3
        J = orc.couplings(L, 99, 5)
        up = np.ones(N, np.int8)
        assert orc.energy(L, J, up) == -int(J.astype(np.int64).sum())
        assert orc.energy(L, J, up) == -3 * N + 2 * orc.n_minus(L, J)
        if L % 2 == 0:
            stag = np.array([1 if (i % L + (i // L) % L + i // (L * L)) % 2 == 0 else -1 for i in range(N)], np.int8)
            assert orc.energy(L, J, stag) == int(J.astype(np.int64).sum())


def test_flip_energy_change_is_12_minus_4u(orc):
    rng = np.random.default_rng(1)
    for L in (2, 3, 4):
        N = L ** 3
        J = orc.couplings(L, 5, 2)
        for _ in range(20):
            S = rng.choice(np.array([-1, 1], np.int8), size=N)
            i = int(rng.integers(N))
            u = orc.unsatisfied(L, J, S, i)
            E0 = orc.energy(L, J, S)
            S2 = S.copy()
            S2[i] = -S2[i]
            assert orc.energy(L, J, S2) - E0 == 12 - 4 * u


def _numpy_energies_L2(J):
    """All 256 energies of an L=2 lattice, evaluated bond by bond."""
    L, N = 2, 8
    states = np.array(list(itertools.product([1, -1], repeat=N)), np.int64)[:, ::-1]
    E = np.zeros(len(states), np.int64)
    for z, y, x in itertools.product(range(L), repeat=3):
        i = site(L, x, y, z)
        for d, (dx, dy, dz) in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            j = site(L, x + dx, y + dy, z + dz)
            E -= J[d * N + i] * states[:, i] * states[:, j]
    return E


@pytest.mark.parametrize("real_id", range(6))
def test_brute_dos_L2(orc, real_id):
    L, N = 2, 8
    J = orc.couplings(L, 20110856, real_id)
    g = orc.brute_dos(L, J)
    eb = orc.e_base(L, J)
    E = _numpy_energies_L2(J.astype(np.int64))
    assert np.all((E - (-3 * N + 2 * orc.n_minus(L, J))) % 4 == 0)
    ref = np.bincount((E - eb) // 4, minlength=len(g))
    assert np.array_equal(ref, g.astype(np.int64))
    assert g.sum() == 2 ** N
    assert np.all(g % 2 == 0)
    # even L: symmetric about E = 0
    levels = eb + 4 * np.arange(len(g))
    for k, e in enumerate(levels):
        if -e >= eb and (-e - eb) % 4 == 0:
            assert g[k] == g[(-e - eb) // 4]
        else:
            assert g[k] == 0


@pytest.fixture(scope="module")
def dos_L3(orc):
    out = []
    for real_id in (0, 1):
        J = orc.couplings(3, 20110856, real_id)
        out.append((J, orc.brute_dos(3, J)))
    return out


def test_brute_dos_L3_invariants(orc, dos_L3):
    L, N = 3, 27
    for J, g in dos_L3:
        assert int(g.sum()) == 2 ** N
        assert np.all(g % 2 == 0)
        # g_J(E) = g_{-J}(-E): flipping every coupling mirrors the spectrum
        Jm = (-J).astype(np.int8)
        gm = orc.brute_dos(L, Jm)
        eb, ebm = orc.e_base(L, J), orc.e_base(L, Jm)
        dos = {eb + 4 * k: int(v) for k, v in enumerate(g) if v}
        dosm = {ebm + 4 * k: int(v) for k, v in enumerate(gm) if v}
        assert dos == {-e: v for e, v in dosm.items()}


def _lnZ(g, eb, beta):
    E = eb + 4 * np.arange(len(g), dtype=np.float64)
    m = g > 0
    a = np.log(g[m].astype(np.float64)) - beta * E[m]
    amax = a.max()
    return amax + math.log(np.exp(a - amax).sum())


def _series_coefficients(g, eb, N, nbonds, orders):
    """Fit F(beta) = ln Z - N ln 2 - nbonds ln cosh(beta) as a polynomial in t = tanh(beta)."""
    betas = np.linspace(0.004, 0.06, 40)
    t = np.tanh(betas)
    F = np.array([_lnZ(g, eb, b) - N * math.log(2) - nbonds * math.log(math.cosh(b)) for b in betas])
    lo = orders[0]
    A = np.stack([t ** k for k in range(lo, lo + 6)], axis=1)
    coef = np.linalg.lstsq(A, F, rcond=None)[0]
    return coef


def test_high_temperature_series_L3(orc, dos_L3):
    """ln Z = N ln 2 + 3N ln cosh b + t^3 sum_lines prod J + t^4 sum_plaquettes prod J + O(t^5).
    At L = 3 the shortest closed loops are the 27 straight lines that wrap around
    the torus (3 bonds) and the 81 elementary plaquettes (4 bonds)."""
    L, N = 3, 27
    for J, g in dos_L3:
        Jd = lambda d, x, y, z: int(J[d * N + site(L, x, y, z)])
        lines = 0
        for d in range(3):
            for a, b in itertools.product(range(L), repeat=2):
                p = 1
                for s in range(L):
                    xyz = [a, b]
                    xyz.insert(d, s)
                    p *= Jd(d, *xyz)
                lines += p
        plaq = 0
        for z, y, x in itertools.product(range(L), repeat=3):
            for d1, d2 in ((0, 1), (1, 2), (0, 2)):
                e1 = [0, 0, 0]; e1[d1] = 1
                e2 = [0, 0, 0]; e2[d2] = 1
                p = Jd(d1, x, y, z) * Jd(d2, x + e1[0], y + e1[1], z + e1[2]) \
                    * Jd(d1, x + e2[0], y + e2[1], z + e2[2]) * Jd(d2, x, y, z)
                plaq += p
        coef = _series_coefficients(g, orc.e_base(L, J), N, 3 * N, (3,))
        assert abs(coef[0] - lines) < 0.05, (coef[:2], lines, plaq)
        assert abs(coef[1] - plaq) < 0.5, (coef[:2], lines, plaq)


def test_high_temperature_series_L2(orc):
    """At L = 2 the neighbours i + e_d and i - e_d coincide, so each such pair is
    joined by two couplings and forms a 2-bond loop: the t^2 coefficient is the
    sum over the 12 pairs of the product of their two couplings."""
    L, N = 2, 8
    for real_id in range(4):
        J = orc.couplings(L, 77, real_id)
        g = orc.brute_dos(L, J)
        a2 = 0
        for z, y, x in itertools.product(range(L), repeat=3):
            for d, e in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
                i = site(L, x, y, z)
                j = site(L, x + e[0], y + e[1], z + e[2])
                if i < j:
                    a2 += int(J[d * N + i]) * int(J[d * N + j])
        coef = _series_coefficients(g, orc.e_base(L, J), N, 3 * N, (2,))
        assert abs(coef[0] - a2) < 0.05, (coef[:2], a2)


def test_sweep_order_is_checkerboard(orc):
    for L in (2, 3, 4, 6):
        o = orc.sweep_order(L)
        N = L ** 3
        assert sorted(o.tolist()) == list(range(N))
        col = [(i % L + (i // L) % L + i // (L * L)) % 2 for i in o]
        n0 = col.count(0)
        assert col == [0] * n0 + [1] * (N - n0)
        assert list(o[:n0]) == sorted(o[:n0]) and list(o[n0:]) == sorted(o[n0:])


def test_coupling_and_spin_bit_layout(orc):
    """Couplings come from word c/32 = output[m&3] of counter (m>>2, real, 0, TAG_J);
    spins from (m>>2, 0, real, walker<<8 | TAG_SPIN). Re-derive a few bits."""
    L, N = 4, 64
    seed = 0x0123456789ABCDEF
    J = orc.couplings(L, seed, 17)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for c in (0, 31, 32, 100, 191):
        m = c // 32
        w = orc.philox([m >> 2, 17, 0, orc.TAG_J], key)[m & 3]
        assert J[c] == (-1 if (int(w) >> (c % 32)) & 1 else 1)
    S = orc.spins(L, seed, 17, 5)
    for i in (0, 33, 63):
        m = i // 32
        w = orc.philox([m >> 2, 0, 17, (5 << 8) | orc.TAG_SPIN], key)[m & 3]
        assert S[i] == (-1 if (int(w) >> (i % 32)) & 1 else 1)
    # about half of the couplings are negative (p = 1/2, Sec. II)
    Jb = np.concatenate([orc.couplings(8, 11, r) for r in range(8)])
    assert abs((Jb < 0).mean() - 0.5) < 0.02
