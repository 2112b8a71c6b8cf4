"""Python binding of libnfm (include/nfm.h): argument marshalling only.

Every step of the sampler runs in the HIP kernels of ``libnfm.so``. PyTorch is
used for the device workspace and the stream. The binding refuses to run when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnfm.so")

NFM_OK, NFM_EINVAL, NFM_ERANGE, NFM_EDEVICE, NFM_ESTATE, NFM_ESIZE = 0, -1, -2, -3, -4, -5
_STATUS = {0: "OK", -1: "EINVAL", -2: "ERANGE", -3: "EDEVICE", -4: "ESTATE", -5: "ESIZE"}


class NfmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def check_device_tensor(t, device, shape, what: str, dtype=None):
    """Refuse (ValueError) a tensor the kernels cannot take as a row-major array of `dtype`
    (default float32) of exactly `shape` on `device` (a torch.device): every pointer handed to
    the library must cover what its kernels read and write."""
    import torch
    dtype = torch.float32 if dtype is None else dtype
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what}: a torch tensor is required, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{what}: dtype {dtype} required, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: shape {tuple(shape)} required, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: a contiguous (row-major) tensor is required")
    if t.device.type != "cuda" or (device is not None and t.device.index != device.index):
        raise ValueError(f"{what}: a tensor on {device} is required, got {t.device}")
    return C.c_void_p(t.data_ptr())


def _sweep_count(n) -> int:
    n = int(n)
    if n < 0:
        raise ValueError(f"sweep count must be >= 0, got {n}")
    return n


class BatchDesc(C.Structure):
    _fields_ = [("n_real", C.c_int32), ("L", C.POINTER(C.c_int32)), ("walkers", C.POINTER(C.c_int32)),
                ("disorder_seed", C.c_uint64), ("walker_seed", C.c_uint64), ("first_real_id", C.c_uint32),
                ("trace_capacity", C.c_int32)]


WALKER_DTYPE = np.dtype([("E", np.int32), ("E_min", np.int32), ("rt_state", np.int32), ("new_min", np.int32),
                         ("rt_count", np.uint64), ("t_first", np.uint64), ("t_last", np.uint64)], align=True)
REAL_DTYPE = np.dtype([("rt_count", np.uint64), ("rt_time", np.uint64), ("E_min", np.int32), ("new_min", np.int32),
                       ("walkers_with_trips", np.int32), ("pad", np.int32), ("reserved", np.uint64)], align=True)

REC_DTYPE = np.dtype([("k_lo", np.int32), ("k_top", np.int32), ("profile", np.int32), ("converged", np.int32),
                      ("iterations", np.int32), ("k_lo_changed", np.int32), ("pl_dE", np.float64),
                      ("pl_alpha", np.float64), ("flatness", np.float64), ("k_seed", np.int32),
                      ("pad", np.int32)], align=True)
WL_DTYPE = np.dtype([("ln_f", np.float64), ("flatness", np.float64), ("stage", np.int32), ("done", np.int32),
                     ("k_top", np.int32), ("updates", np.int32)], align=True)
RT_SUMMARY_DTYPE = np.dtype([("tau_pop", np.float64), ("trips", np.uint64), ("n_used", np.int32),
                             ("n_censored", np.int32)], align=True)
PROFILE_FLAT, PROFILE_POWER, PROFILE_INVK = 0, 1, 2
TUNING_FIELDS = ("speculate", "sweeps_per_launch", "schedule", "waves_per_cu", "hist", "ws")
TUNE_RESULT_DTYPE = np.dtype([("tuning", np.int32, (6,)), ("attempts_per_s", np.float64)], align=True)

class Frechet(C.Structure):
    """nfm_frechet: parameters (mu, beta, xi) of Eq. (9)."""
    _fields_ = [("mu", C.c_double), ("beta", C.c_double), ("xi", C.c_double)]

    def as_tuple(self):
        return (self.mu, self.beta, self.xi)


class Ratio(C.Structure):
    """nfm_ratio: relative performance with jackknife errors and the two fits."""
    _fields_ = [("r_pop", C.c_double), ("r_pop_err", C.c_double), ("r_eps", C.c_double),
                ("r_eps_err", C.c_double), ("fit_m", Frechet), ("fit_ref", Frechet),
                ("blocks", C.c_int32), ("pad", C.c_int32)]


_lib = None


def lib():
    """Load libnfm.so; raise if it is missing (there is no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libnfm.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_size_t
    sig = {
        "nfm_workspace_bytes": (i32, [C.POINTER(BatchDesc), C.POINTER(sz)]),
        "nfm_create": (i32, [C.POINTER(vp), C.POINTER(BatchDesc), vp, sz, C.c_int, vp]),
        "nfm_destroy": (None, [vp]),
        "nfm_last_error": (C.c_char_p, [vp]),
        "nfm_n_real": (i32, [vp]),
        "nfm_n_walkers": (i64, [vp]),
        "nfm_levels": (i32, [vp, i32]),
        "nfm_e_base": (i32, [vp, i32]),
        "nfm_level_offset": (i64, [vp, i32]),
        "nfm_levels_total": (i64, [vp]),
        "nfm_walker_offset": (i64, [vp, i32]),
        "nfm_sweep_counter": (u64, [vp]),
        "nfm_init_couplings": (i32, [vp]),
        "nfm_set_couplings": (i32, [vp, i32, i32, vp]),
        "nfm_get_couplings": (i32, [vp, i32, i32, vp]),
        "nfm_init_spins": (i32, [vp]),
        "nfm_set_spins": (i32, [vp, i64, i64, vp]),
        "nfm_get_spins": (i32, [vp, i64, i64, vp]),
        "nfm_compute_energies": (i32, [vp]),
        "nfm_set_thresholds": (i32, [vp, i32, vp, i32, i32]),
        "nfm_get_thresholds": (i32, [vp, i32, vp, C.POINTER(i32), C.POINTER(i32)]),
        "nfm_set_weights_lnw": (i32, [vp, vp, vp, vp]),
        "nfm_set_rt_bounds": (i32, [vp, i32, i32, i32]),
        "nfm_run_sweeps": (i32, [vp, u64]),
        "nfm_read_histograms": (i32, [vp, vp, C.c_int]),
        "nfm_reset_histograms": (i32, [vp]),
        "nfm_read_walkers": (i32, [vp, vp]),
        "nfm_read_realizations": (i32, [vp, vp]),
        "nfm_read_trace": (i32, [vp, vp, C.POINTER(i32)]),
        "nfm_reset_trace": (i32, [vp]),
        "nfm_trace_config": (i32, [vp, i64, i64, i32]),
        "nfm_trace_range": (i32, [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32)]),
        "nfm_sync": (i32, [vp]),
        "nfm_checkpoint_bytes": (i32, [vp, C.POINTER(sz)]),
        "nfm_last_kernel": (C.c_char_p, [vp]),
        "nfm_checkpoint": (i32, [vp, vp, sz]),
        "nfm_restore": (i32, [vp, vp, sz]),
        "nfm_set_histograms": (i32, [vp, vp]),
        "nfm_reset_round_trips": (i32, [vp]),
        "nfm_stuck_walkers": (i32, [vp, u64, vp, C.POINTER(i64)]),
        "nfm_rec_init": (i32, [vp, i32, C.c_double, C.c_double]),
        "nfm_rec_update": (i32, [vp, C.c_double, vp]),
        "nfm_rec_production": (i32, [vp, i32, C.c_double, C.c_double]),
        "nfm_wl_init": (i32, [vp, C.c_double]),
        "nfm_wl_update": (i32, [vp, C.c_double, C.c_double, vp]),
        "nfm_wl_get": (i32, [vp, i32, vp, vp, vp]),
        "nfm_wl_to_rec": (i32, [vp, i32, C.c_double, C.c_double]),
        "nfm_rec_read_info": (i32, [vp, vp]),
        "nfm_rec_get_state": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, vp]),
        "nfm_rec_set_state": (i32, [vp, i32, vp, vp, vp, vp, vp, vp]),
        "nfm_set_tuning": (i32, [vp, vp]),
        "nfm_get_tuning": (i32, [vp, vp]),
        "nfm_pt_init": (i32, [vp, i32, vp]),
        "nfm_pt_set_temps": (i32, [vp, i32, vp]),
        "nfm_pt_get_temps": (i32, [vp, i32, vp]),
        "nfm_pt_get_tables": (i32, [vp, i32, vp, vp, C.POINTER(i32), C.POINTER(i32)]),
        "nfm_pt_adapt": (i32, [vp, C.c_double, C.c_double, vp, C.POINTER(i32)]),
        "nfm_pt_run_sweeps": (i32, [vp, u64]),
        "nfm_pt_read_slots": (i32, [vp, vp]),
        "nfm_pt_set_slots": (i32, [vp, vp]),
        "nfm_pt_read_exchanges": (i32, [vp, vp]),
        "nfm_rt_stats": (i32, [vp, i32, i32, u64, vp, vp]),
        "nfm_autotune": (i32, [vp, i32, C.c_char_p, vp, i32, C.POINTER(i32), vp]),
        "nfm_rec_seed": (i32, [vp, vp, vp]),
        "nfm_rec_seed_grid": (i32, [vp, vp, vp]),
        "nfm_set_canonical": (i32, [vp, C.c_double]),
        "nfm_rec_targets": (i32, [vp, vp, vp]),
        "nfm_features": (i32, [vp, vp]),
    }
    dbl = C.c_double
    sig.update({
        "nfm_frechet_cdf": (dbl, [C.POINTER(Frechet), dbl]),
        "nfm_frechet_quantile": (dbl, [C.POINTER(Frechet), dbl]),
        "nfm_frechet_mean": (dbl, [C.POINTER(Frechet)]),
        "nfm_frechet_quantile_mean": (dbl, [C.POINTER(Frechet), dbl]),
        "nfm_upper_gamma": (dbl, [dbl, dbl]),
        "nfm_frechet_fit": (i32, [vp, i64, i32, C.POINTER(Frechet), C.POINTER(dbl)]),
        "nfm_relative_performance": (i32, [vp, vp, i64, dbl, i32, i32, C.POINTER(Ratio)]),
        "nfm_frechet_fit_jackknife": (i32, [vp, i64, i32, i32, C.POINTER(Frechet), C.POINTER(Frechet),
                                            C.POINTER(i32)]),
        "nfm_running_mean": (i32, [vp, i64, vp]),
        "nfm_frechet_ks": (i32, [C.POINTER(Frechet), vp, i64, C.POINTER(dbl)]),
        "nfm_stats_last_error": (C.c_char_p, []),
    })
    f32 = C.c_float
    sig.update({
        "nfm_mlp_n_params": (i32, []),
        "nfm_mlp_workspace_bytes": (i32, [i32, C.POINTER(sz)]),
        "nfm_mlp_create": (i32, [C.POINTER(vp), i32, vp, sz, C.c_int, vp]),
        "nfm_mlp_destroy": (None, [vp]),
        "nfm_mlp_last_error": (C.c_char_p, [vp]),
        "nfm_mlp_init": (i32, [vp, u64]),
        "nfm_mlp_set_params": (i32, [vp, vp, vp]),
        "nfm_mlp_get_params": (i32, [vp, vp, vp]),
        "nfm_mlp_get_grads": (i32, [vp, vp]),
        "nfm_mlp_forward": (i32, [vp, vp, i32, vp]),
        "nfm_mlp_loss_grad": (i32, [vp, vp, vp, vp, i32, vp]),
        "nfm_mlp_adam": (i32, [vp, f32, f32, f32, f32]),
        "nfm_mlp_train_step": (i32, [vp, vp, vp, vp, i32, f32]),
        "nfm_mlp_last_loss": (i32, [vp, vp]),
        "nfm_mlp_to_bf16": (i32, [vp]),
        "nfm_mlp_infer_bf16": (i32, [vp, vp, i32, vp]),
        "nfm_mlp_infer_bf16_noalloc": (i32, [vp, vp, i32, vp]),
    })
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _desc(Ls: Sequence[int], walkers: Sequence[int], disorder_seed: int, walker_seed: int,
          first_real_id: int, trace_capacity: int):
    La = np.ascontiguousarray(Ls, np.int32).reshape(-1)
    Wa = np.ascontiguousarray(walkers, np.int32).reshape(-1)
    if len(La) != len(Wa):
        # the library reads n_real entries of both arrays: refuse before it reads past one
        raise NfmError(NFM_EINVAL, f"batch description: {len(La)} sizes but {len(Wa)} walker counts")
    d = BatchDesc(len(La), La.ctypes.data_as(C.POINTER(C.c_int32)), Wa.ctypes.data_as(C.POINTER(C.c_int32)),
                  disorder_seed, walker_seed, first_real_id, trace_capacity)
    return d, (La, Wa)


def workspace_bytes(Ls, walkers, trace_capacity=0) -> int:
    d, keep = _desc(Ls, walkers, 0, 0, 0, trace_capacity)
    n = C.c_size_t()
    st = lib().nfm_workspace_bytes(C.byref(d), C.byref(n))
    if st != NFM_OK:
        raise NfmError(st, "invalid batch description")
    return n.value


def pack_couplings(J: np.ndarray, L: int) -> np.ndarray:
    """ABI coupling words of one realization from +-1 couplings J[d*N + i]."""
    N = L ** 3
    JW = (N + 31) // 32
    bits = (np.asarray(J).reshape(3, N) < 0).astype(np.uint32)
    out = np.zeros((3, JW * 32), np.uint32)
    out[:, :N] = bits
    w = out.reshape(3, JW, 32) << np.arange(32, dtype=np.uint32)
    return np.bitwise_or.reduce(w, axis=2).reshape(-1).astype(np.uint32)


def unpack_couplings(words: np.ndarray, L: int) -> np.ndarray:
    N = L ** 3
    JW = (N + 31) // 32
    w = np.asarray(words, np.uint32).reshape(3, JW, 1)
    bits = ((w >> np.arange(32, dtype=np.uint32)) & 1).reshape(3, JW * 32)[:, :N]
    return np.where(bits.reshape(-1) == 1, -1, 1).astype(np.int8)


class Batch:
    """One context of libnfm over a torch-allocated device workspace."""

    def __init__(self, Ls: Sequence[int], walkers: Sequence[int], disorder_seed: int = 0, walker_seed: int = 0,
                 first_real_id: int = 0, trace_capacity: int = 0, device: int = 0, stream=None):
        import torch
        self._lib = lib()
        self.Ls = np.ascontiguousarray(Ls, np.int32)
        self.walkers = np.ascontiguousarray(walkers, np.int32)
        self.trace_capacity = trace_capacity
        d, self._keep = _desc(self.Ls, self.walkers, disorder_seed, walker_seed, first_real_id, trace_capacity)
        n = C.c_size_t()
        self._check(self._lib.nfm_workspace_bytes(C.byref(d), C.byref(n)), "workspace size")
        self.device = torch.device("cuda", device)
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        ctx = C.c_void_p()
        self._check(self._lib.nfm_create(C.byref(ctx), C.byref(d), C.c_void_p(aligned), n.value, device,
                                         C.c_void_p(stream.cuda_stream)), "create")
        self.ctx = ctx

    def _check(self, st, what):
        if st != NFM_OK:
            msg = self._lib.nfm_last_error(self.ctx).decode() if getattr(self, "ctx", None) else what
            raise NfmError(st, f"{what}: {msg}")

    def close(self):
        if getattr(self, "ctx", None):
            self._lib.nfm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # geometry
    @property
    def n_real(self) -> int:
        return int(self._lib.nfm_n_real(self.ctx))

    @property
    def n_walkers(self) -> int:
        return int(self._lib.nfm_n_walkers(self.ctx))

    def levels(self, r: int) -> int:
        return int(self._lib.nfm_levels(self.ctx, r))

    def e_base(self, r: int) -> int:
        return int(self._lib.nfm_e_base(self.ctx, r))

    def level_offset(self, r: int) -> int:
        return int(self._lib.nfm_level_offset(self.ctx, r))

    @property
    def levels_total(self) -> int:
        return int(self._lib.nfm_levels_total(self.ctx))

    def walker_offset(self, r: int) -> int:
        return int(self._lib.nfm_walker_offset(self.ctx, r))

    @property
    def sweep_counter(self) -> int:
        return int(self._lib.nfm_sweep_counter(self.ctx))

    # couplings and spins
    def init_couplings(self):
        self._check(self._lib.nfm_init_couplings(self.ctx), "init_couplings")

    def set_couplings(self, r0: int, words: np.ndarray):
        words = np.ascontiguousarray(words, np.uint32)
        L = int(self.Ls[r0])
        per = 3 * ((L ** 3 + 31) // 32)
        count = words.size // per
        self._check(self._lib.nfm_set_couplings(self.ctx, r0, count, words.ctypes.data), "set_couplings")

    def get_couplings(self, r0: int, count: int = 1) -> np.ndarray:
        n = sum(3 * ((int(self.Ls[r]) ** 3 + 31) // 32) for r in range(r0, r0 + count))
        out = np.zeros(n, np.uint32)
        self._check(self._lib.nfm_get_couplings(self.ctx, r0, count, out.ctypes.data), "get_couplings")
        return out

    def init_spins(self):
        self._check(self._lib.nfm_init_spins(self.ctx), "init_spins")

    def _walker_sizes(self, w0: int, count: int):
        sizes = []
        for r in range(self.n_real):
            off, W, N = self.walker_offset(r), int(self.walkers[r]), int(self.Ls[r]) ** 3
            lo, hi = max(w0, off), min(w0 + count, off + W)
            if hi > lo:
                sizes.append((hi - lo) * N)
        return sum(sizes)

    def set_spins(self, w0: int, S: np.ndarray):
        S = np.ascontiguousarray(S, np.int8)
        if S.ndim == 1:   # walkers back to back, each with the N of its realization
            count, used, w = 0, 0, w0
            while used < S.size:
                used += int(self.Ls[self._real_of(w)]) ** 3
                count += 1
                w += 1
            if used != S.size:
                raise ValueError("set_spins: array length does not end on a walker boundary")
        else:
            count = S.shape[0]
        if self._walker_sizes(w0, count) != S.size:
            raise ValueError("set_spins: array size does not match the walkers' lattice sizes")
        self._check(self._lib.nfm_set_spins(self.ctx, w0, count, S.ctypes.data), "set_spins")

    def get_spins(self, w0: int, count: int) -> np.ndarray:
        out = np.zeros(self._walker_sizes(w0, count), np.int8)
        self._check(self._lib.nfm_get_spins(self.ctx, w0, count, out.ctypes.data), "get_spins")
        return out

    def _real_of(self, w: int) -> int:
        for r in range(self.n_real):
            if self.walker_offset(r) <= w < self.walker_offset(r) + int(self.walkers[r]):
                return r
        raise IndexError(w)

    def compute_energies(self):
        self._check(self._lib.nfm_compute_energies(self.ctx), "compute_energies")

    # tables
    def set_thresholds(self, r: int, thr: np.ndarray, row0: int):
        thr = np.ascontiguousarray(thr, np.uint32).reshape(-1, 8)
        self._check(self._lib.nfm_set_thresholds(self.ctx, r, thr.ctypes.data, row0, thr.shape[0]), "set_thresholds")

    def get_thresholds(self, r: int):
        row0, rows = C.c_int32(), C.c_int32()
        self._check(self._lib.nfm_get_thresholds(self.ctx, r, None, C.byref(row0), C.byref(rows)), "get_thresholds")
        out = np.zeros((max(rows.value, 1), 8), np.uint32)
        self._check(self._lib.nfm_get_thresholds(self.ctx, r, out.ctypes.data, C.byref(row0), C.byref(rows)),
                    "get_thresholds")
        return out[:rows.value], row0.value

    def set_weights_lnw(self, lnw: np.ndarray, k_lo: Sequence[int], k_top: Sequence[int]):
        lnw = np.ascontiguousarray(lnw, np.float64)
        assert lnw.size == self.levels_total
        klo = np.ascontiguousarray(k_lo, np.int32)
        ktop = np.ascontiguousarray(k_top, np.int32)
        self._check(self._lib.nfm_set_weights_lnw(self.ctx, lnw.ctypes.data, klo.ctypes.data, ktop.ctypes.data),
                    "set_weights_lnw")

    def set_rt_bounds(self, r: int, e_bot: int, e_top: int):
        self._check(self._lib.nfm_set_rt_bounds(self.ctx, r, e_bot, e_top), "set_rt_bounds")

    # sampling and read-back
    def run_sweeps(self, n: int):
        self._check(self._lib.nfm_run_sweeps(self.ctx, _sweep_count(n)), "run_sweeps")

    def read_histograms(self, reset: bool = False) -> np.ndarray:
        out = np.zeros(self.levels_total, np.uint64)
        self._check(self._lib.nfm_read_histograms(self.ctx, out.ctypes.data, 1 if reset else 0), "read_histograms")
        return out

    def reset_histograms(self):
        self._check(self._lib.nfm_reset_histograms(self.ctx), "reset_histograms")

    def read_walkers(self) -> np.ndarray:
        out = np.zeros(self.n_walkers, WALKER_DTYPE)
        self._check(self._lib.nfm_read_walkers(self.ctx, out.ctypes.data), "read_walkers")
        return out

    def read_realizations(self) -> np.ndarray:
        out = np.zeros(self.n_real, REAL_DTYPE)
        self._check(self._lib.nfm_read_realizations(self.ctx, out.ctypes.data), "read_realizations")
        return out

    def trace_range(self):
        """(first walker, walkers, capacity) of the trace in effect."""
        w0, nw, cap = C.c_int64(), C.c_int64(), C.c_int32()
        self._check(self._lib.nfm_trace_range(self.ctx, C.byref(w0), C.byref(nw), C.byref(cap)), "trace_range")
        return w0.value, nw.value, cap.value

    def trace_config(self, walker_begin: int, count: int, capacity: int):
        """Trace walkers [walker_begin, walker_begin + count) for up to `capacity` sweeps from now on."""
        self._check(self._lib.nfm_trace_config(self.ctx, int(walker_begin), int(count), int(capacity)), "trace_config")

    def read_trace(self):
        """The traced walkers' energies, [walkers of the traced range, sweeps traced so far]."""
        n = C.c_int32()
        _, nw, cap = self.trace_range()
        out = np.zeros((nw, max(cap, 0)), np.int32)
        self._check(self._lib.nfm_read_trace(self.ctx, out.ctypes.data if out.size else None, C.byref(n)),
                    "read_trace")
        return out[:, :n.value]

    def reset_trace(self):
        self._check(self._lib.nfm_reset_trace(self.ctx), "reset_trace")

    def sync(self):
        self._check(self._lib.nfm_sync(self.ctx), "sync")

    def last_kernel(self) -> str:
        """The sweep kernel form the last launch used (nfm_last_kernel)."""
        return self._lib.nfm_last_kernel(self.ctx).decode()

    def checkpoint(self) -> np.ndarray:
        """The whole state of the context as a host byte array (nfm_checkpoint)."""
        n = C.c_size_t()
        self._check(self._lib.nfm_checkpoint_bytes(self.ctx, C.byref(n)), "checkpoint_bytes")
        blob = np.empty(n.value, np.uint8)
        self._check(self._lib.nfm_checkpoint(self.ctx, blob.ctypes.data, n.value), "checkpoint")
        return blob

    def restore(self, blob: np.ndarray):
        """Load a checkpoint of a batch with the same description (nfm_restore)."""
        blob = np.ascontiguousarray(blob, np.uint8)
        self._check(self._lib.nfm_restore(self.ctx, blob.ctypes.data, blob.size), "restore")

    # weight recursion
    def set_histograms(self, H: np.ndarray):
        H = np.ascontiguousarray(H, np.uint64)
        assert H.size == self.levels_total
        self._check(self._lib.nfm_set_histograms(self.ctx, H.ctypes.data), "set_histograms")

    def reset_round_trips(self):
        self._check(self._lib.nfm_reset_round_trips(self.ctx), "reset_round_trips")

    def stuck_walkers(self, window_sweeps: int, flags=None) -> int:
        """Walkers without a completed round trip in the last window_sweeps sweeps
        (nfm_stuck_walkers): their number; flags, if given, a uint8 device tensor of n_walkers
        entries, receives 1 for each flagged walker."""
        import torch
        window = int(window_sweeps)
        if window < 0:
            raise ValueError("stuck_walkers: window_sweeps must be >= 0")
        ptr = C.c_void_p(None)
        if flags is not None:
            ptr = check_device_tensor(flags, self.device, (self.n_walkers,), "stuck_walkers: flags", torch.uint8)
        n = C.c_int64()
        self._check(self._lib.nfm_stuck_walkers(self.ctx, window, ptr, C.byref(n)), "stuck_walkers")
        return int(n.value)

    def rec_init(self, profile: int = PROFILE_FLAT, pl_dE: float = 1.0, pl_alpha: float = 0.0):
        self._check(self._lib.nfm_rec_init(self.ctx, profile, pl_dE, pl_alpha), "rec_init")

    def rec_update(self, f_tol: float = 0.5) -> np.ndarray:
        info = np.zeros(self.n_real, REC_DTYPE)
        self._check(self._lib.nfm_rec_update(self.ctx, f_tol, info.ctypes.data), "rec_update")
        return info

    def rec_production(self, profile: int, pl_dE: float = 96.0, pl_alpha: float = -3.6):
        self._check(self._lib.nfm_rec_production(self.ctx, profile, pl_dE, pl_alpha), "rec_production")

    # Wang-Landau estimate
    def wl_init(self, ln_f0: float = 1.0):
        self._check(self._lib.nfm_wl_init(self.ctx, ln_f0), "wl_init")

    def wl_update(self, flat_tol: float = 0.8, ln_f_final: float = 1e-4) -> np.ndarray:
        info = np.zeros(self.n_real, WL_DTYPE)
        self._check(self._lib.nfm_wl_update(self.ctx, flat_tol, ln_f_final, info.ctypes.data), "wl_update")
        return info

    def wl_get(self, r: int):
        """(ln g, stage histogram, info) of realization r (3N/2 + 1 entries each)."""
        n = 3 * int(self.Ls[r]) ** 3 // 2 + 1
        lng = np.zeros(n, np.float64)
        hst = np.zeros(n, np.uint64)
        info = np.zeros(1, WL_DTYPE)
        self._check(self._lib.nfm_wl_get(self.ctx, r, lng.ctypes.data, hst.ctypes.data, info.ctypes.data), "wl_get")
        return lng, hst, info[0]

    def wl_to_rec(self, profile: int = PROFILE_FLAT, pl_dE: float = 1.0, pl_alpha: float = 0.0):
        self._check(self._lib.nfm_wl_to_rec(self.ctx, profile, pl_dE, pl_alpha), "wl_to_rec")

    def rec_read_info(self) -> np.ndarray:
        info = np.zeros(self.n_real, REC_DTYPE)
        self._check(self._lib.nfm_rec_read_info(self.ctx, info.ctypes.data), "rec_read_info")
        return info

    def rec_get_state(self, r: int) -> dict:
        n = 3 * int(self.Ls[r]) ** 3 // 2 + 1
        out = {k: np.zeros(n, np.float64) for k in ("b", "p", "S", "lnP", "lnW")}
        out["visited"] = np.zeros(n, np.uint8)
        info = np.zeros(1, REC_DTYPE)
        self._check(self._lib.nfm_rec_get_state(self.ctx, r, out["b"].ctypes.data, out["p"].ctypes.data,
                                                out["S"].ctypes.data, out["lnP"].ctypes.data,
                                                out["lnW"].ctypes.data, out["visited"].ctypes.data,
                                                info.ctypes.data), "rec_get_state")
        out["info"] = info[0]
        return out

    def rec_set_state(self, r: int, b, p, lnP, lnW, visited, k_lo: int, k_top: int, profile: int = PROFILE_FLAT,
                      pl_dE: float = 1.0, pl_alpha: float = 0.0, k_seed: int = -1):
        n = 3 * int(self.Ls[r]) ** 3 // 2 + 1
        arr = [np.zeros(n, np.float64) for _ in range(4)]
        for a, v in zip(arr, (b, p, lnP, lnW)):
            a[:len(v)] = v
        vis = np.zeros(n, np.uint8)
        vis[:len(visited)] = visited
        info = np.zeros(1, REC_DTYPE)
        info["k_lo"], info["k_top"], info["profile"] = k_lo, k_top, profile
        info["pl_dE"], info["pl_alpha"] = pl_dE, pl_alpha
        info["k_seed"] = k_seed
        self._check(self._lib.nfm_rec_set_state(self.ctx, r, arr[0].ctypes.data, arr[1].ctypes.data,
                                                arr[2].ctypes.data, arr[3].ctypes.data, vis.ctypes.data,
                                                info.ctypes.data), "rec_set_state")

    # launch tuning
    def set_tuning(self, speculate: int = -1, sweeps_per_launch: int = 0, schedule: int = 0, waves_per_cu: int = 0,
                   hist: int = 0, ws: int = 0):
        t = np.array([speculate, sweeps_per_launch, schedule, waves_per_cu, hist, ws], np.int32)
        self._check(self._lib.nfm_set_tuning(self.ctx, t.ctypes.data), "set_tuning")

    def get_tuning(self) -> dict:
        t = np.zeros(len(TUNING_FIELDS), np.int32)
        self._check(self._lib.nfm_get_tuning(self.ctx, t.ctypes.data), "get_tuning")
        return dict(zip(TUNING_FIELDS, (int(x) for x in t)))

    def autotune(self, calib_sweeps: int = 256, cache_path: Optional[str] = None, max_results: int = 128):
        """Time the candidate launch configurations on this batch (state restored afterwards),
        apply the fastest. Returns (best tuning dict, list of (tuning dict, attempts/s))."""
        res = np.zeros(max_results, TUNE_RESULT_DTYPE)
        n = C.c_int32()
        best = np.zeros(len(TUNING_FIELDS), np.int32)
        path = cache_path.encode() if cache_path else None
        self._check(self._lib.nfm_autotune(self.ctx, calib_sweeps, path, res.ctypes.data if max_results else None,
                                           max_results, C.byref(n), best.ctypes.data), "autotune")
        table = [(dict(zip(TUNING_FIELDS, (int(x) for x in r["tuning"]))), float(r["attempts_per_s"]))
                 for r in res[:n.value]]
        return dict(zip(TUNING_FIELDS, (int(x) for x in best))), table

    # parallel tempering
    def pt_init(self, temps):
        T = np.ascontiguousarray(temps, np.float64)
        self._check(self._lib.nfm_pt_init(self.ctx, len(T), T.ctypes.data), "pt_init")

    def pt_tables(self, r: int = 0):
        """(metro [M, 8], swap [M-1, D]) of realization r, as the kernel computes them."""
        M, D = C.c_int32(), C.c_int32()
        self._check(self._lib.nfm_pt_get_tables(self.ctx, r, None, None, C.byref(M), C.byref(D)), "pt_get_tables")
        metro = np.zeros((M.value, 8), np.uint32)
        swap = np.zeros((max(M.value - 1, 0), D.value), np.uint32)
        self._check(self._lib.nfm_pt_get_tables(self.ctx, r, metro.ctypes.data, swap.ctypes.data, C.byref(M),
                                                C.byref(D)), "pt_get_tables")
        return metro, swap

    def pt_set_temps(self, r: int, temps):
        T = np.ascontiguousarray(temps, np.float64)
        self._check(self._lib.nfm_pt_set_temps(self.ctx, r, T.ctypes.data), "pt_set_temps")

    def pt_temps(self, r: int, M: int) -> np.ndarray:
        T = np.zeros(M, np.float64)
        self._check(self._lib.nfm_pt_get_temps(self.ctx, r, T.ctypes.data), "pt_get_temps")
        return T

    def pt_adapt(self, M: int, rate_lo: float = 0.4, rate_hi: float = 0.6):
        """One adaptation step of every realization's temperatures toward a constant exchange
        rate. Returns (rates [n_real, M-1] measured since the last step, pairs outside the band)."""
        rates = np.zeros((self.n_real, M - 1), np.float64)
        n_out = C.c_int32()
        self._check(self._lib.nfm_pt_adapt(self.ctx, rate_lo, rate_hi, rates.ctypes.data, C.byref(n_out)),
                    "pt_adapt")
        return rates, n_out.value

    def pt_run_sweeps(self, n: int):
        self._check(self._lib.nfm_pt_run_sweeps(self.ctx, _sweep_count(n)), "pt_run_sweeps")

    def pt_slots(self) -> np.ndarray:
        out = np.zeros(self.n_walkers, np.int32)
        self._check(self._lib.nfm_pt_read_slots(self.ctx, out.ctypes.data), "pt_read_slots")
        return out

    def pt_set_slots(self, slots):
        sl = np.ascontiguousarray(slots, np.int32)
        self._check(self._lib.nfm_pt_set_slots(self.ctx, sl.ctypes.data), "pt_set_slots")

    def pt_exchanges(self, M: int) -> np.ndarray:
        """Accepted exchanges, [n_sets, M - 1], n_sets = (n_walkers / 64) floor(64 / M)."""
        out = np.zeros(((self.n_walkers // 64) * (64 // M), M - 1), np.uint64)
        self._check(self._lib.nfm_pt_read_exchanges(self.ctx, out.ctypes.data), "pt_read_exchanges")
        return out

    # round-trip statistics
    def rt_stats(self, r0: int = 0, count: Optional[int] = None, min_trips: int = 1):
        """(tau per realization [count] in sweeps, NaN = censored; summary record)."""
        count = self.n_real - r0 if count is None else count
        tau = np.zeros(count, np.float64)
        summ = np.zeros(1, RT_SUMMARY_DTYPE)
        self._check(self._lib.nfm_rt_stats(self.ctx, r0, count, min_trips, tau.ctypes.data, summ.ctypes.data),
                    "rt_stats")
        return tau, summ[0]

    # learned seeding
    def rec_seed(self, b_levels, k_seed):
        """Seeded prior: b_levels (levels_total doubles, by level offset), k_seed per realization
        (-1 = leave it plain)."""
        bl = np.ascontiguousarray(b_levels, np.float64)
        ks = np.ascontiguousarray(k_seed, np.int32)
        self._check(self._lib.nfm_rec_seed(self.ctx, bl.ctypes.data, ks.ctypes.data), "rec_seed")

    def rec_seed_grid(self, curves) -> np.ndarray:
        """Seeded prior from device curves (torch float32 [n_real, 256] on this GPU); returns k_seed
        per realization (-1: rejected, plain start kept)."""
        ks = np.zeros(self.n_real, np.int32)
        pc = check_device_tensor(curves, self.device, (self.n_real, 256), "rec_seed_grid curves")
        self._check(self._lib.nfm_rec_seed_grid(self.ctx, pc, ks.ctypes.data),
                    "rec_seed_grid")
        return ks

    def rec_targets(self):
        """(y, mask) torch float32 [n_real, 256] on this GPU from the current estimate."""
        import torch
        y = torch.empty((self.n_real, 256), dtype=torch.float32, device=self.device)
        m = torch.empty_like(y)
        self._check(self._lib.nfm_rec_targets(self.ctx, C.c_void_p(y.data_ptr()), C.c_void_p(m.data_ptr())),
                    "rec_targets")
        return y, m

    def set_canonical(self, T: float):
        self._check(self._lib.nfm_set_canonical(self.ctx, T), "set_canonical")

    def features(self, out=None):
        """Inputs of the seeding model into a torch float32 [n_real, 81] tensor on this GPU."""
        import torch
        if out is None:
            out = torch.empty((self.n_real, 81), dtype=torch.float32, device=self.device)
        po = check_device_tensor(out, self.device, (self.n_real, 81), "features out")
        self._check(self._lib.nfm_features(self.ctx, po), "features")
        return out


class Mlp:
    """The weight-seeding network over a torch-allocated device workspace (nfm_mlp_*)."""

    N_IN, N_OUT = 81, 256

    def __init__(self, batch_max: int = 256, device: int = 0, stream=None):
        import torch
        self._lib = lib()
        self.batch_max = batch_max
        n = C.c_size_t()
        st = self._lib.nfm_mlp_workspace_bytes(batch_max, C.byref(n))
        if st != NFM_OK:
            raise NfmError(st, "mlp workspace size")
        self.device = torch.device("cuda", device)
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        aligned = (self._ws.data_ptr() + 255) // 256 * 256
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        ctx = C.c_void_p()
        st = self._lib.nfm_mlp_create(C.byref(ctx), batch_max, C.c_void_p(aligned), n.value, device,
                                      C.c_void_p(stream.cuda_stream))
        if st != NFM_OK:
            raise NfmError(st, "mlp create")
        self.ctx = ctx
        self.n_params = int(self._lib.nfm_mlp_n_params())

    def _check(self, st, what):
        if st != NFM_OK:
            raise NfmError(st, f"{what}: {self._lib.nfm_mlp_last_error(self.ctx).decode()}")

    def close(self):
        if getattr(self, "ctx", None):
            self._lib.nfm_mlp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, seed: int):
        self._check(self._lib.nfm_mlp_init(self.ctx, seed), "init")

    def set_params(self, params=None, norm=None):
        p = None if params is None else np.ascontiguousarray(params, np.float32)
        q = None if norm is None else np.ascontiguousarray(norm, np.float32)
        self._check(self._lib.nfm_mlp_set_params(self.ctx, None if p is None else p.ctypes.data,
                                                 None if q is None else q.ctypes.data), "set_params")

    def get_params(self):
        p = np.zeros(self.n_params, np.float32)
        q = np.zeros((2, self.N_IN), np.float32)
        self._check(self._lib.nfm_mlp_get_params(self.ctx, p.ctypes.data, q.ctypes.data), "get_params")
        return p, q

    def get_grads(self):
        g = np.zeros(self.n_params, np.float32)
        self._check(self._lib.nfm_mlp_get_grads(self.ctx, g.ctypes.data), "get_grads")
        return g

    def _rows(self, x, what) -> int:
        B = int(x.shape[0]) if hasattr(x, "shape") and len(x.shape) >= 1 else -1
        if not 1 <= B <= self.batch_max:
            raise ValueError(f"{what}: between 1 and {self.batch_max} rows required, got {B}")
        return B

    def _x(self, x, what):
        B = self._rows(x, what)
        return B, check_device_tensor(x, self.device, (B, self.N_IN), what + " x")

    def _y(self, t, B, what):
        return check_device_tensor(t, self.device, (B, self.N_OUT), what)

    def forward(self, x, out=None):
        import torch
        B, px = self._x(x, "forward")
        if out is None:
            out = torch.empty((B, self.N_OUT), dtype=torch.float32, device=self.device)
        self._check(self._lib.nfm_mlp_forward(self.ctx, px, B, self._y(out, B, "forward out")), "forward")
        return out

    def loss_grad(self, x, t, mask) -> float:
        loss = C.c_float()
        B, px = self._x(x, "loss_grad")
        self._check(self._lib.nfm_mlp_loss_grad(self.ctx, px, self._y(t, B, "loss_grad t"),
                                                self._y(mask, B, "loss_grad mask"), B, C.byref(loss)), "loss_grad")
        return float(loss.value)

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self._lib.nfm_mlp_adam(self.ctx, lr, beta1, beta2, eps), "adam")

    def train_step(self, x, t, mask, lr=1e-3):
        B, px = self._x(x, "train_step")
        self._check(self._lib.nfm_mlp_train_step(self.ctx, px, self._y(t, B, "train_step t"),
                                                 self._y(mask, B, "train_step mask"), B, lr), "train_step")

    def last_loss(self) -> float:
        loss = C.c_float()
        self._check(self._lib.nfm_mlp_last_loss(self.ctx, C.byref(loss)), "last_loss")
        return float(loss.value)

    def to_bf16(self):
        self._check(self._lib.nfm_mlp_to_bf16(self.ctx), "to_bf16")

    def infer_bf16(self, x, out=None):
        import torch
        B, px = self._x(x, "infer_bf16")
        if out is None:
            out = torch.empty((B, self.N_OUT), dtype=torch.float32, device=self.device)
        self._check(self._lib.nfm_mlp_infer_bf16(self.ctx, px, B, self._y(out, B, "infer_bf16 out")), "infer_bf16")
        return out

    NOALLOC_ROWS = 1024

    def infer_bf16_noalloc(self, x, out):
        """nfm_mlp_infer_bf16_noalloc: the same inference with the library's static scratch (at most
        NOALLOC_ROWS rows, any batch_max); the caller passes the output tensor [B, 256]."""
        B = int(x.shape[0]) if hasattr(x, "shape") and len(x.shape) >= 1 else -1
        px = check_device_tensor(x, self.device, (B, self.N_IN), "infer_bf16_noalloc x")
        py = check_device_tensor(out, self.device, (B, self.N_OUT), "infer_bf16_noalloc out")
        self._check(self._lib.nfm_mlp_infer_bf16_noalloc(self.ctx, px, B, py), "infer_bf16_noalloc")
        return out


# --------------------------------------------------------------------------- round-trip statistics
# Host functions of the library (Secs. IV, V); times are per-realization mean round-trip times.

def _frechet(params) -> Frechet:
    mu, beta, xi = params
    return Frechet(float(mu), float(beta), float(xi))


def frechet_cdf(params, tau: float) -> float:
    """F(tau) of Eq. (9) for params = (mu, beta, xi)."""
    return lib().nfm_frechet_cdf(C.byref(_frechet(params)), float(tau))


def frechet_quantile(params, p: float) -> float:
    """Q(p) of Eq. (13)."""
    return lib().nfm_frechet_quantile(C.byref(_frechet(params)), float(p))


def frechet_mean(params) -> float:
    """Eq. (11); inf for xi >= 1."""
    return lib().nfm_frechet_mean(C.byref(_frechet(params)))


def frechet_quantile_mean(params, eps: float) -> float:
    """Eq. (14) in closed form."""
    return lib().nfm_frechet_quantile_mean(C.byref(_frechet(params)), float(eps))


def upper_gamma(a: float, x: float) -> float:
    """Gamma(a, x) for real a, x > 0."""
    return lib().nfm_upper_gamma(float(a), float(x))


def _times(t) -> np.ndarray:
    return np.ascontiguousarray(t, dtype=np.float64)


def frechet_fit(tau, method: int = 0):
    """Fit of Eq. (9) to times tau: method 0 maximum likelihood, 1 least squares on the
    empirical CDF. Returns ((mu, beta, xi), objective)."""
    t = _times(tau)
    out, obj = Frechet(), C.c_double()
    st = lib().nfm_frechet_fit(t.ctypes.data, len(t), int(method), C.byref(out), C.byref(obj))
    if st != 0:
        raise NfmError(st, "frechet_fit: " + lib().nfm_stats_last_error().decode())
    return out.as_tuple(), obj.value


def relative_performance(tau_m, tau_ref, eps: float = 1e-4, method: int = 0, blocks: int = 0) -> dict:
    """r_pop and r_eps (Table I) of method m against the reference, with jackknife errors."""
    a, b = _times(tau_m), _times(tau_ref)
    if len(a) != len(b):
        raise ValueError("relative_performance: paired samples of equal length")
    out = Ratio()
    st = lib().nfm_relative_performance(a.ctypes.data, b.ctypes.data, len(a), float(eps), int(method),
                                        int(blocks), C.byref(out))
    if st != 0:
        raise NfmError(st, "relative_performance: " + lib().nfm_stats_last_error().decode())
    return {"r_pop": out.r_pop, "r_pop_err": out.r_pop_err, "r_eps": out.r_eps, "r_eps_err": out.r_eps_err,
            "fit_m": out.fit_m.as_tuple(), "fit_ref": out.fit_ref.as_tuple(), "blocks": out.blocks}


def frechet_fit_jackknife(tau, method: int = 0, blocks: int = 0):
    """Fit of Eq. (9) and the delete-a-block jackknife errors of its parameters (Fig. 4: the shape
    xi with jackknife errors). Returns ((mu, beta, xi), (err_mu, err_beta, err_xi), blocks)."""
    t = _times(tau)
    fit, err, B = Frechet(), Frechet(), C.c_int32()
    st = lib().nfm_frechet_fit_jackknife(t.ctypes.data, len(t), int(method), int(blocks), C.byref(fit), C.byref(err),
                                         C.byref(B))
    if st != 0:
        raise NfmError(st, "frechet_fit_jackknife: " + lib().nfm_stats_last_error().decode())
    return fit.as_tuple(), err.as_tuple(), B.value


def running_mean(tau) -> np.ndarray:
    """Eq. (12) over the realizations in the given order: out[i] = mean of tau[0..i]."""
    t = _times(tau)
    out = np.zeros(len(t), np.float64)
    st = lib().nfm_running_mean(t.ctypes.data, len(t), out.ctypes.data)
    if st != 0:
        raise NfmError(st, "running_mean: " + lib().nfm_stats_last_error().decode())
    return out


def frechet_ks(params, tau) -> float:
    """sup |F_n - F| between the empirical CDF of the times and Eq. (9) with these parameters."""
    t = _times(tau)
    d = C.c_double()
    st = lib().nfm_frechet_ks(C.byref(_frechet(params)), t.ctypes.data, len(t), C.byref(d))
    if st != 0:
        raise NfmError(st, "frechet_ks: " + lib().nfm_stats_last_error().decode())
    return d.value
