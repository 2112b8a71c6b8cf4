"""Python view of the CPU oracle (TEST INFRASTRUCTURE).

The oracle is the plain sequential model that the GPU library is checked
against. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import this module. The product path never does.

The arithmetic lives in ``nfm_oracle.c``; this module only marshals numpy
arrays and strings the per-iteration steps of the weight recursion together
in the order the method prescribes (weights -> sample -> update, Sec. II of
Muller/Schnabel/Janke, arXiv:2011.08560).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import math

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nfm_oracle.c")
LIB = os.path.join(HERE, "libnfm_oracle.so")

PROFILE_FLAT, PROFILE_POWER, PROFILE_INVK = 0, 1, 2
TAG_ACC, TAG_SPIN, TAG_J, TAG_PT, TAG_SWAP = 1, 2, 3, 4, 5

WALKER_DTYPE = np.dtype(
    [
        ("E", np.int32),
        ("E_min", np.int32),
        ("rt_state", np.int32),
        ("new_min", np.int32),
        ("rt_count", np.uint64),
        ("t_first", np.uint64),
        ("t_last", np.uint64),
    ],
    align=True,
)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, so fp64 sums match the
    operation order written in the source)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = np.ctypeslib.ndpointer
        i32, u32, u64, i64, dbl = C.c_int32, C.c_uint32, C.c_uint64, C.c_int64, C.c_double
        L.orc_philox4x32_10.argtypes = [P(np.uint32), P(np.uint32), P(np.uint32)]
        L.orc_n_minus.argtypes = [i32, P(np.int8)]
        L.orc_n_minus.restype = i32
        L.orc_e_base.argtypes = [i32, P(np.int8)]
        L.orc_e_base.restype = i32
        L.orc_n_levels.argtypes = [i32, P(np.int8)]
        L.orc_n_levels.restype = i32
        L.orc_sweep_order.argtypes = [i32, P(np.int32)]
        L.orc_gen_couplings.argtypes = [i32, u64, u32, P(np.int8)]
        L.orc_gen_spins.argtypes = [i32, u64, u32, u32, P(np.int8)]
        L.orc_energy.argtypes = [i32, P(np.int8), P(np.int8)]
        L.orc_energy.restype = i32
        L.orc_unsatisfied.argtypes = [i32, P(np.int8), P(np.int8), i32]
        L.orc_unsatisfied.restype = i32
        L.orc_table_rows.argtypes = [i32, i32, i32, C.POINTER(i32)]
        L.orc_table_rows.restype = i32
        L.orc_build_thresholds.argtypes = [i32, P(np.float64), i32, i32, P(np.uint32),
                                           C.POINTER(i32), C.POINTER(i32)]
        L.orc_build_thresholds.restype = i32
        L.orc_track.argtypes = [C.c_void_p, i32, i32, i32, u64]
        L.orc_muca_sweeps.argtypes = [i32, P(np.int8), P(np.int8), C.c_void_p, P(np.uint32), i32, i32,
                                      i32, i32, u64, u32, u32, u64, u64, C.c_void_p, C.c_void_p, i32]
        L.orc_muca_sweeps.restype = i32
        L.orc_metropolis_accept.argtypes = [u32, u32]
        L.orc_metropolis_accept.restype = i32
        L.orc_pow_bin.argtypes = [dbl, i32]
        L.orc_pow_bin.restype = dbl
        L.orc_pt_swap_q.argtypes = [dbl, dbl]
        L.orc_pt_swap_q.restype = dbl
        L.orc_brute_dos.argtypes = [i32, P(np.int8), P(np.uint64)]
        L.orc_brute_dos.restype = i32
        L.orc_power_profile.argtypes = [dbl, dbl, dbl, dbl]
        L.orc_power_profile.restype = dbl
        L.orc_rec_weights.argtypes = [i32, i32, i32, i32, i32, dbl, dbl, P(np.float64),
                                      P(np.float64), P(np.float64), P(np.float64)]
        L.orc_rec_update.argtypes = [i32, i32, i32, i32, P(np.float64), P(np.float64), P(np.uint64),
                                     P(np.float64), P(np.float64), P(np.uint8), C.POINTER(i32),
                                     C.POINTER(dbl)]
        L.orc_rec_weights_ext.argtypes = [i32, i32, i32, i32, i32, i32, dbl, dbl, P(np.float64),
                                          P(np.float64), P(np.float64), P(np.float64)]
        L.orc_rec_update_ext.argtypes = [i32, i32, i32, i32, i32, i32, P(np.float64), P(np.float64), P(np.uint64),
                                         P(np.float64), P(np.float64), P(np.uint8), C.POINTER(i32),
                                         C.POINTER(dbl)]
        L.orc_seed_from_grid.argtypes = [i32, i32, i32, P(np.float32), P(np.float64)]
        L.orc_seed_from_grid.restype = i32
        L.orc_features.argtypes = [i32, P(np.int8), P(np.float64)]
        L.orc_hist_bins.argtypes = [i32, i32, i32, P(np.uint64), P(np.float64)]
        L.orc_pt_metro_table.argtypes = [i32, P(np.float64), P(np.uint32)]
        L.orc_pt_swap_table.argtypes = [i32, P(np.float64), i32, C.c_void_p]
        L.orc_pt_swap_table.restype = i32
        L.orc_pt_sweeps.argtypes = [i32, P(np.int8), i32, P(np.int8), C.c_void_p, P(np.int32), P(np.uint32),
                                    P(np.uint32), i32, i32, i32, u64, u32, u32, u32, u64, u64, C.c_void_p,
                                    C.c_void_p, i32]
        L.orc_pt_sweeps.restype = i32
        _lib = L
    return _lib


# --------------------------------------------------------------------------- basic wrappers

def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.ascontiguousarray(ctr, np.uint32), np.ascontiguousarray(key, np.uint32), out)
    return out


def couplings(L: int, seed: int, real_id: int) -> np.ndarray:
    J = np.zeros(3 * L ** 3, np.int8)
    lib().orc_gen_couplings(L, seed, real_id, J)
    return J


def spins(L: int, seed: int, real_id: int, walker: int) -> np.ndarray:
    S = np.zeros(L ** 3, np.int8)
    lib().orc_gen_spins(L, seed, real_id, walker, S)
    return S


def energy(L: int, J: np.ndarray, S: np.ndarray) -> int:
    return int(lib().orc_energy(L, np.ascontiguousarray(J, np.int8), np.ascontiguousarray(S, np.int8)))


def unsatisfied(L: int, J: np.ndarray, S: np.ndarray, i: int) -> int:
    return int(lib().orc_unsatisfied(L, J, S, i))


def e_base(L: int, J: np.ndarray) -> int:
    return int(lib().orc_e_base(L, J))


def n_levels(L: int, J: np.ndarray) -> int:
    return int(lib().orc_n_levels(L, J))


def n_minus(L: int, J: np.ndarray) -> int:
    return int(lib().orc_n_minus(L, J))


def sweep_order(L: int) -> np.ndarray:
    o = np.zeros(L ** 3, np.int32)
    lib().orc_sweep_order(L, o)
    return o


def level_of(E: int, eb: int) -> int:
    return (E - eb) // 4


def table_rows(K: int, k_lo: int, k_top: int):
    row0 = C.c_int32()
    rows = lib().orc_table_rows(K, k_lo, k_top, C.byref(row0))
    return row0.value, rows


def build_thresholds(K: int, lnw_levels: np.ndarray, k_lo: int, k_top: int):
    """lnw_levels: log-weights on levels k_lo..k_top. Returns (thr[rows, 8], row0)."""
    lnw = np.ascontiguousarray(lnw_levels, np.float64)
    assert lnw.shape[0] == k_top - k_lo + 1
    row0, rows = table_rows(K, k_lo, k_top)
    thr = np.zeros(rows * 8, np.uint32)
    r0, nr = C.c_int32(), C.c_int32()
    rc = lib().orc_build_thresholds(K, lnw, k_lo, k_top, thr, C.byref(r0), C.byref(nr))
    if rc != 0:
        raise ValueError("bad level range")
    return thr.reshape(nr.value, 8), r0.value


def new_walkers(n: int, E0) -> np.ndarray:
    w = np.zeros(n, WALKER_DTYPE)
    w["E"] = E0
    w["E_min"] = E0
    return w


def track(w: np.ndarray, E: int, e_bot: int, e_top: int, tau: int) -> None:
    lib().orc_track(w.ctypes.data, E, e_bot, e_top, tau)


def metropolis_accept(r, thr):
    """Acceptance of an attempt with random word r under stored threshold thr (Eq. (2),
    probabilities quantised down to multiples of 2^-32 with 2^-32 as the least)."""
    return bool(lib().orc_metropolis_accept(int(r), int(thr)))


def muca_sweeps(L, J, S, w, thr, row0, e_bot, e_top, walker_seed, real_id, walker,
                t0, n_sweeps, hist=None, trace=None, check_energy=False):
    """Run n_sweeps for one walker in place (S: int8[N], w: one-element WALKER_DTYPE array)."""
    thr = np.ascontiguousarray(thr, np.uint32).reshape(-1)
    rows = thr.shape[0] // 8
    rc = lib().orc_muca_sweeps(L, J, S, w.ctypes.data, thr, row0, rows, e_bot, e_top,
                               walker_seed, real_id, walker, t0, n_sweeps,
                               None if hist is None else hist.ctypes.data,
                               None if trace is None else trace.ctypes.data,
                               1 if check_energy else 0)
    if rc == -1:
        raise AssertionError("incremental energy disagrees with recomputation")
    if rc != 0:
        raise RuntimeError("oracle sweep failed")


def brute_dos(L: int, J: np.ndarray) -> np.ndarray:
    g = np.zeros(n_levels(L, J), np.uint64)
    if lib().orc_brute_dos(L, J, g) != 0:
        raise ValueError("lattice too large for enumeration")
    return g


def power_profile(E, E_g, dE, alpha) -> float:
    return float(lib().orc_power_profile(E, E_g, dE, alpha))


def rec_weights(K, eb, k_lo, k_top, profile, pl_dE, pl_alpha, b):
    S = np.zeros(K, np.float64)
    lnP = np.zeros(K, np.float64)
    lnW = np.zeros(K, np.float64)
    lib().orc_rec_weights(K, eb, k_lo, k_top, profile, pl_dE, pl_alpha,
                          np.ascontiguousarray(b, np.float64), S, lnP, lnW)
    return S, lnP, lnW


def rec_update(K, k_lo_used, k_top, k_min_seen, lnW_used, lnP_used, H, b, p, visited):
    """In-place update of b, p, visited. Returns (k_lo_new, flatness)."""
    kl = C.c_int32()
    fl = C.c_double()
    lib().orc_rec_update(K, k_lo_used, k_top, k_min_seen, lnW_used, lnP_used,
                         np.ascontiguousarray(H, np.uint64), b, p, visited, C.byref(kl), C.byref(fl))
    return kl.value, fl.value


def rec_weights_ext(K, eb, k_lo, k_top, k_low, profile, pl_dE, pl_alpha, b):
    S = np.zeros(K, np.float64)
    lnP = np.zeros(K, np.float64)
    lnW = np.zeros(K, np.float64)
    lib().orc_rec_weights_ext(K, eb, k_lo, k_top, k_low, profile, pl_dE, pl_alpha,
                              np.ascontiguousarray(b, np.float64), S, lnP, lnW)
    return S, lnP, lnW


def rec_update_ext(K, k_lo_used, k_top, k_low_used, seeded, k_min_seen, lnW_used, lnP_used, H, b, p, visited):
    kl = C.c_int32()
    fl = C.c_double()
    lib().orc_rec_update_ext(K, k_lo_used, k_top, k_low_used, 1 if seeded else 0, k_min_seen, lnW_used, lnP_used,
                             np.ascontiguousarray(H, np.uint64), b, p, visited, C.byref(kl), C.byref(fl))
    return kl.value, fl.value


def seed_from_grid(N, eb, k_top, y, b):
    """Fill b on [k_s, k_top) from a 256-point curve (in place); returns k_s or -1 (rejected)."""
    return int(lib().orc_seed_from_grid(N, eb, k_top, np.ascontiguousarray(y, np.float32), b))


def features(L, J) -> np.ndarray:
    out = np.zeros(16, np.float64)
    lib().orc_features(L, J, out)
    return out


def hist_bins(K, eb, N, H) -> np.ndarray:
    out = np.zeros(64, np.float64)
    lib().orc_hist_bins(K, eb, N, np.ascontiguousarray(H, np.uint64), out)
    return out


# --------------------------------------------------------------------------- weight iteration

@dataclass
class Realization:
    """One disorder realization with its walkers, as the oracle sees it."""
    L: int
    J: np.ndarray
    real_id: int
    walker_seed: int
    S: np.ndarray          # int8 [W, N]
    w: np.ndarray          # WALKER_DTYPE [W]
    t: int = 0             # absolute sweep counter

    @property
    def N(self):
        return self.L ** 3

    @property
    def eb(self):
        return e_base(self.L, self.J)

    @property
    def K(self):
        return n_levels(self.L, self.J)

    @property
    def k_top(self):
        """Lowest level with E >= 0 (the 'highest energy' end, Sec. III)."""
        return -(self.eb) // 4 if (-self.eb) % 4 == 0 else -(self.eb) // 4 + 1


def make_realization(L, disorder_seed, real_id, walker_seed, walkers) -> Realization:
    J = couplings(L, disorder_seed, real_id)
    S = np.stack([spins(L, walker_seed, real_id, w) for w in range(walkers)])
    E0 = np.array([energy(L, J, S[w]) for w in range(walkers)], np.int32)
    return Realization(L, J, real_id, walker_seed, S, new_walkers(walkers, E0))


def sample(rz: Realization, thr, row0, e_bot, e_top, n_sweeps, trace=False):
    """Run every walker n_sweeps; returns (pooled histogram, traces or None)."""
    H = np.zeros(rz.K, np.uint64)
    tr = np.zeros((rz.S.shape[0], n_sweeps), np.int32) if trace else None
    for wk in range(rz.S.shape[0]):
        ws = rz.w[wk:wk + 1].copy()
        Sw = rz.S[wk].copy()
        muca_sweeps(rz.L, rz.J, Sw, ws, thr, row0, e_bot, e_top, rz.walker_seed, rz.real_id, wk,
                    rz.t, n_sweeps, hist=H, trace=None if tr is None else tr[wk])
        rz.S[wk] = Sw
        rz.w[wk] = ws[0]
    rz.t += n_sweeps
    return H, tr


@dataclass
class RecursionState:
    b: np.ndarray
    p: np.ndarray
    visited: np.ndarray
    k_lo: int
    k_top: int


def recursion_init(rz: Realization) -> RecursionState:
    K = rz.K
    k_lo = min(int(level_of(int(e), rz.eb)) for e in rz.w["E_min"])
    return RecursionState(np.zeros(K), np.zeros(K), np.zeros(K, np.uint8), min(k_lo, rz.k_top), rz.k_top)


def weight_iterations(rz: Realization, st: RecursionState, n_iter: int, n_sweeps: int,
                      profile=PROFILE_FLAT, pl_dE=1.0, pl_alpha=0.0, f_tol=0.5, stop=True, k_seed=-1):
    """The weight iteration (Sec. II): build weights from the DOS estimate and the
    target profile, sample, update the estimate; stop at the first iteration whose
    histogram is flat to f_tol with no new minimum. With k_seed >= 0 the estimate's steps
    b on [k_seed, k_lo) are a seeded prior (see seed_from_grid): they continue the weights
    below k_lo and are kept when those levels are first reached. Returns a list of
    per-iteration records (iteration, k_lo, flatness, converged)."""
    log = []
    seeded = k_seed >= 0
    for it in range(n_iter):
        k_low = min(k_seed, st.k_lo) if seeded else st.k_lo
        S, lnP, lnW = rec_weights_ext(rz.K, rz.eb, st.k_lo, st.k_top, k_low, profile, pl_dE, pl_alpha, st.b)
        thr, row0 = build_thresholds(rz.K, lnW[k_low:st.k_top + 1], k_low, st.k_top)
        e_lo = rz.eb + 4 * st.k_lo
        H, _ = sample(rz, thr, row0, e_lo, 0, n_sweeps)
        k_min = int(level_of(int(rz.w["E_min"].min()), rz.eb))
        k_lo_old = st.k_lo
        st.k_lo, flat = rec_update_ext(rz.K, st.k_lo, st.k_top, k_low, seeded, min(k_min, st.k_lo), lnW, lnP, H,
                                       st.b, st.p, st.visited)
        conv = flat >= f_tol and st.k_lo == k_lo_old
        log.append((it, st.k_lo, flat, conv))
        if conv and stop:
            break
    return log


def production_weights(rz: Realization, st: RecursionState, kind: str, pl_dE=96.0, pl_alpha=-3.6):
    """Production ensembles from the final estimate (Sec. II): flat lnW = -S,
    power law -S + ln P_SH, 1/k -S + (S - ln sum exp S). Returns lnW on levels."""
    prof = {"flat": PROFILE_FLAT, "power": PROFILE_POWER, "invk": PROFILE_INVK}[kind]
    S, lnP, lnW = rec_weights(rz.K, rz.eb, st.k_lo, st.k_top, prof, pl_dE, pl_alpha, st.b)
    return lnW


# --------------------------------------------------------------------------- parallel tempering

# --------------------------------------------------------------------------- Wang-Landau (batched)

def wl_k_top(eb: int) -> int:
    """Lowest level with E >= 0: the estimate lives on [0, k_top]."""
    return (-eb + 3) // 4


@dataclass
class WangLandau:
    """Batched Wang-Landau state of one realization: ln g on [0, k_top] (zero elsewhere), the
    histogram of the current stage, ln f, halvings so far, done flag, last flatness."""
    lng: np.ndarray
    hst: np.ndarray
    ln_f: float
    k_top: int
    stage: int = 0
    done: bool = False
    flatness: float = 0.0
    updates: int = 0


def wl_init(K: int, eb: int, ln_f0: float) -> WangLandau:
    return WangLandau(np.zeros(K), np.zeros(K, np.uint64), float(ln_f0), wl_k_top(eb))


def wl_update(st: WangLandau, H, flat_tol: float, ln_f_final: float) -> None:
    """One step: ln g(k) += ln f H(k) and Hs(k) += H(k) on k <= k_top; flatness = min/mean of Hs
    over the levels it visited; a flat stage halves ln f and clears Hs; done once ln f < final."""
    if st.done:
        return
    for k in range(st.k_top + 1):
        h = int(H[k])
        if h:
            st.lng[k] += st.ln_f * float(h)
        st.hst[k] += np.uint64(h)
    vis = [int(x) for x in st.hst[:st.k_top + 1] if x > 0]
    flat = (float(min(vis)) / (float(sum(vis)) / float(len(vis)))) if vis else 0.0
    st.flatness = flat
    st.updates += 1
    if flat >= flat_tol:
        st.ln_f = 0.5 * st.ln_f
        st.stage += 1
        st.hst[:] = 0
        if st.ln_f < ln_f_final:
            st.done = True


def wl_thresholds(st: WangLandau, K: int):
    """Tables of the weights lnW = -ln g on [0, k_top]."""
    return build_thresholds(K, -st.lng[:st.k_top + 1], 0, st.k_top)


def wl_to_rec_steps(st: WangLandau):
    """(k_lo, b) handed to the recursion: visited = ln g > 0, k_lo = the lowest visited level,
    b(k) = ln g(k+1) - ln g(k) on [k_lo, k_top), zero elsewhere."""
    vis = [k for k in range(st.k_top + 1) if st.lng[k] > 0.0]
    k_lo = min(vis) if vis else st.k_top
    b = np.zeros(len(st.lng))
    for k in range(k_lo, st.k_top):
        b[k] = st.lng[k + 1] - st.lng[k]
    return k_lo, b


def pt_temperatures(M: int, t_min: float = 0.2, t_max: float = 2.0) -> np.ndarray:
    """Geometric temperature ladder T_s = t_min (t_max/t_min)^(s/(M-1))."""
    return np.array([t_min * (t_max / t_min) ** (s / (M - 1)) for s in range(M)], np.float64)


def pt_metro_table(T) -> np.ndarray:
    T = np.ascontiguousarray(T, np.float64)
    thr = np.zeros(len(T) * 8, np.uint32)
    lib().orc_pt_metro_table(len(T), T, thr)
    return thr.reshape(len(T), 8)


def pow_bin(q: float, d: int) -> float:
    return lib().orc_pow_bin(float(q), int(d))


def pt_swap_q(T_lo: float, T_hi: float) -> float:
    return lib().orc_pt_swap_q(float(T_lo), float(T_hi))


def pt_swap_table(T, d_cap: int) -> np.ndarray:
    """(M-1) x D exchange thresholds, entry [s][d-1] for d = (E_{s+1} - E_s)/4."""
    T = np.ascontiguousarray(T, np.float64)
    D = lib().orc_pt_swap_table(len(T), T, d_cap, None)
    thr = np.zeros((len(T) - 1) * D, np.uint32)
    lib().orc_pt_swap_table(len(T), T, d_cap, thr.ctypes.data)
    return thr.reshape(len(T) - 1, D)


@dataclass
class PTSet:
    """One parallel-tempering set: M configurations of one realization."""
    L: int
    J: np.ndarray
    real_id: int
    walker_seed: int
    set_index: int
    walker0: int           # walker index of configuration 0
    S: np.ndarray          # int8 [M, N]
    w: np.ndarray          # WALKER_DTYPE [M]
    slot: np.ndarray       # int32 [M], temperature slot of each configuration
    t: int = 0


def pt_set_walker0(M, set_index):
    """Walker index of configuration 0 of a set: every group of 64 walkers holds floor(64/M)
    sets of M consecutive walkers (the rest of the group idles)."""
    spw = 64 // M
    return 64 * (set_index // spw) + M * (set_index % spw)


def make_pt_set(L, disorder_seed, real_id, walker_seed, M, set_index=0) -> PTSet:
    """Configurations start from the spins of the set's walkers walker0 .. walker0+M-1;
    configuration c starts at slot c."""
    J = couplings(L, disorder_seed, real_id)
    w0 = pt_set_walker0(M, set_index)
    ws = [w0 + c for c in range(M)]
    S = np.stack([spins(L, walker_seed, real_id, w) for w in ws])
    E0 = np.array([energy(L, J, S[c]) for c in range(M)], np.int32)
    return PTSet(L, J, real_id, walker_seed, set_index, w0, S, new_walkers(M, E0), np.arange(M, dtype=np.int32))


def pt_exchange_rates(acc_sets, t0, t1, M):
    """Acceptance rate of each pair (s, s+1) of a realization from the accepted exchanges of its
    sets ([n_sets, M-1]) over sweeps t0 <= t < t1: pair s is attempted once per set on every sweep
    with t = s (mod 2)."""
    acc = np.asarray(acc_sets, dtype=np.float64)
    n_sets = acc.shape[0]
    rates = np.zeros(M - 1)
    for s in range(M - 1):
        attempts = sum(1 for t in range(t0, t1) if t % 2 == s % 2)
        rates[s] = acc[:, s].sum() / (n_sets * attempts)
    return rates


def pt_adapt_step(T, rates):
    """One step of the temperature adaptation toward a constant exchange rate (a reading of the
    protocol the paper adopts, whose update it does not print): with gaps g_s = 1/T_s - 1/T_{s+1},
    g_s <- g_s f_s, f_s = (-ln A_s)^(-1/4) limited to [1/2, 2] (A_s clamped to [1e-6, 1 - 1e-12]),
    then all gaps rescaled to their old sum so that T_0 and T_{M-1} stay."""
    beta = [1.0 / float(x) for x in T]
    M = len(beta)
    span = beta[0] - beta[M - 1]
    gaps, total = [], 0.0
    for s in range(M - 1):
        a = min(max(float(rates[s]), 1e-6), 1.0 - 1e-12)
        f = min(max((-math.log(a)) ** -0.25, 0.5), 2.0)
        g = (beta[s] - beta[s + 1]) * f
        gaps.append(g)
        total += g
    new = list(beta)
    for s in range(M - 2):
        new[s + 1] = new[s] - gaps[s] * (span / total)
    new[M - 1] = beta[M - 1]
    return np.array([1.0 / b for b in new])


def pt_sweeps(ps: PTSet, metro, swap, e_bot, e_top, n_sweeps, swap_acc=None, trace=False, check_energy=False):
    """Advance a PT set by n_sweeps in place; returns the traces (M x n_sweeps) or None."""
    M = ps.S.shape[0]
    metro = np.ascontiguousarray(metro, np.uint32).reshape(-1)
    swap = np.ascontiguousarray(swap, np.uint32)
    D = swap.shape[1]
    tr = np.zeros((M, n_sweeps), np.int32) if trace else None
    S = np.ascontiguousarray(ps.S)
    rc = lib().orc_pt_sweeps(ps.L, ps.J, M, S, ps.w.ctypes.data, ps.slot, metro, swap.reshape(-1), D,
                             e_bot, e_top, ps.walker_seed, ps.real_id, ps.set_index, ps.walker0, ps.t, n_sweeps,
                             None if swap_acc is None else swap_acc.ctypes.data,
                             None if tr is None else tr.ctypes.data, 1 if check_energy else 0)
    if rc == -1:
        raise AssertionError("incremental energy disagrees with recomputation")
    if rc != 0:
        raise RuntimeError("oracle PT sweep failed")
    ps.S = S
    ps.t += n_sweeps
    return tr


# --------------------------------------------------------------------------- round-trip statistics

def rt_tau(rt_count, t_first, t_last, N: int, min_trips: int = 1):
    """Round-trip time of one realization (Sec. III), pooled over its walkers: the summed
    time of completed trips, from each walker's first arrival at the top to its last
    completed trip, over the number of trips, in sweeps (attempts / N). Returns
    (tau, trips, censored); censored (tau = nan) when fewer than min_trips trips."""
    rt_count = np.asarray(rt_count, np.uint64)
    done = rt_count > 0
    trips = int(rt_count.sum())
    time = int((np.asarray(t_last, np.uint64)[done] - np.asarray(t_first, np.uint64)[done]).sum())
    if trips < max(1, min_trips):
        return float("nan"), trips, True
    return time / trips / N, trips, False


def rt_population(taus):
    """tau_pop: mean of the uncensored per-realization round-trip times."""
    t = np.asarray(taus, np.float64)
    t = t[~np.isnan(t)]
    return float(t.sum() / len(t)) if len(t) else float("nan")


# --------------------------------------------------------------------------- seeding targets

def rec_targets(N, eb, k_lo, k_top, S):
    """Targets of the seeding model from an estimate S (by level, S(k_top) = 0): y_j = S(e_j N)/N on
    e_j = -2 + 2j/255, linear between levels; mask 1 where e_j N >= E(k_lo)."""
    y = np.zeros(256)
    m = np.zeros(256)
    E_lo, E_top = eb + 4 * k_lo, eb + 4 * k_top
    for j in range(256):
        E = (-2.0 + 2.0 * j / 255.0) * N
        if E < E_lo:
            continue
        if E >= E_top:
            v = S[k_top]
        else:
            t = (E - eb) / 4.0
            k = min(max(int(np.floor(t)), k_lo), k_top - 1)
            v = S[k] + (t - k) * (S[k + 1] - S[k])
        y[j] = v / N
        m[j] = 1.0
    return y, m
