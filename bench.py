"""Benchmark of the multicanonical sampler on one MI355X.

Workload (default): 1024 disorder realizations of the L = 6 bimodal EA spin glass,
64 walkers each, power-law-target weight iteration (Sec. II of Muller, Schnabel,
Janke); one step is one pass of the hot path over the batch: S sweeps of every
walker (per-attempt minimum/round-trip bookkeeping, per-sweep histograms), then the
per-realization reduction of the walker statistics. Synthetic seeded disorder.

Prints ONE JSON line (rank 0): spin-flip attempts per second of the whole job, the
roofline of the sweep kernel (VALU-issue bound) and the CPU oracle's rate on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic integer lane-operations per spin-flip attempt (see the design notes):
# Philox4x32-10 share 10 (2.5 rounds x (2 wide products + 2 three-input xors)),
# neighbour count 1, table address 2, acceptance 2, spin/energy update 2,
# bookkeeping check 1.
ALG_OPS_PER_ATTEMPT = 18.0
# MI355X integer VALU peak: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (one lane-op per cycle).
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9

CONFIGS = {
    # name: (L, realizations, walkers per realization, sweeps per step)
    "c2": (6, 1024, 64, 100_000),
    "c3": (8, 4096, 64, 10_000),
    "c1": (4, 32, 64, 10_000),
}


def gaussian_dos_lnw(L: int, K: int, eb: int) -> np.ndarray:
    """Multicanonical log-weights of a Gaussian approximation of the density of states,
    ln g(E) ~ N ln 2 - E^2/(6N) (the high-temperature form for 3N bonds): lnW = E^2/(6N)."""
    N = L ** 3
    E = eb + 4 * np.arange(K, dtype=np.float64)
    return E * E / (6.0 * N)


def setup(nfm, L, R, W, seed=20110856):
    b = nfm.Batch([L] * R, [W] * R, disorder_seed=seed, walker_seed=seed + 1, first_real_id=0)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    lnw = np.zeros(b.levels_total)
    klo, ktop = [], []
    for r in range(R):
        K, eb = b.levels(r), b.e_base(r)
        off = b.level_offset(r)
        lnw[off:off + K] = gaussian_dos_lnw(L, K, eb)
        k_top = (-eb + 3) // 4
        k_lo = max(0, (int(-1.85 * L ** 3) - eb) // 4)
        klo.append(k_lo)
        ktop.append(k_top)
    b.set_weights_lnw(lnw, klo, ktop)
    for r in range(R):
        b.set_rt_bounds(r, int(-1.6 * L ** 3), 0)
    return b, lnw, klo, ktop


def _oracle_worker(args):
    L, seed, rid, walkers, sweeps, thr, row0, e_bot = args
    from oracle import oracle as orc
    J = orc.couplings(L, seed, rid)
    t0 = time.perf_counter()
    n = 0
    for wk in walkers:
        s = orc.spins(L, seed + 1, rid, wk)
        w = orc.new_walkers(1, orc.energy(L, J, s))
        orc.muca_sweeps(L, J, s, w, thr, row0, e_bot, 0, seed + 1, rid, wk, 0, sweeps)
        n += sweeps * L ** 3
    return n, time.perf_counter() - t0


def cpu_baseline(b, L, lnw, klo, ktop, seconds_target=15.0):
    """The oracle as it stands, one process per core over disjoint walkers of the same
    realizations and weights, on a bounded sample (about seconds_target of wall time)."""
    from oracle import oracle as orc
    cores = max(1, min(16, os.cpu_count() or 1))
    R = min(8, b.n_real)
    tasks = []
    probe_sweeps = 20
    # rate probe on one core to size the sample
    J = orc.couplings(L, 20110856, 0)
    K, eb = orc.n_levels(L, J), orc.e_base(L, J)
    thr, row0 = orc.build_thresholds(K, lnw[b.level_offset(0) + klo[0]:b.level_offset(0) + ktop[0] + 1], klo[0], ktop[0])
    n, dt = _oracle_worker((L, 20110856, 0, [0], probe_sweeps, thr, row0, int(-1.6 * L ** 3)))
    per_core = n / dt
    sweeps = max(10, int(seconds_target * per_core / (L ** 3) / 8))  # 8 walkers per task
    for r in range(R):
        J = orc.couplings(L, 20110856, r)
        K, eb = orc.n_levels(L, J), orc.e_base(L, J)
        off = b.level_offset(r)
        thr, row0 = orc.build_thresholds(K, lnw[off + klo[r]:off + ktop[r] + 1], klo[r], ktop[r])
        for chunk in range(max(1, cores // R)):
            tasks.append((L, 20110856, r, list(range(chunk * 8, chunk * 8 + 8)), sweeps, thr, row0,
                          int(-1.6 * L ** 3)))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_worker, tasks)
    wall = time.perf_counter() - t0
    total = sum(r[0] for r in res)
    return {"value": total / wall, "unit": "spin-flip attempts/s", "cores": cores, "kind": "oracle",
            "sample": f"L={L}, {len(tasks)} tasks x 8 walkers x {sweeps} sweeps over {R} realizations "
                      f"({total:.3g} attempts, {wall:.1f} s wall, {cores} processes)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--sweeps", type=int, default=0, help="sweeps per step (default: the config's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(realizations are independent: shard them across processes, one per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2011_08560_amd import nfm

    L, R, W, S = CONFIGS[args.config]
    if args.sweeps:
        S = args.sweeps
    b, lnw, klo, ktop = setup(nfm, L, R, W)
    stream = torch.cuda.current_stream()
    attempts_per_step = R * W * S * L ** 3
    launches_per_step = math.ceil(S / 1024)

    for _ in range(args.warmup):
        b.run_sweeps(S)
        b.read_realizations()
    torch.cuda.synchronize()
    trips0 = int(b.read_realizations()["rt_count"].sum())

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        b.run_sweeps(S)
        ev[k][1].record(stream)
        b.read_realizations()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    trips = int(b.read_realizations()["rt_count"].sum()) - trips0
    kernel_ms = sum(s.elapsed_time(e) for s, e in ev)
    avg_launch_s = kernel_ms / 1e3 / (args.steps * launches_per_step)
    attempts_per_launch = attempts_per_step / launches_per_step
    achieved = ALG_OPS_PER_ATTEMPT * attempts_per_launch / avg_launch_s / 1e12
    peak = PEAK_LANE_OPS / 1e12

    line = {
        "metric": "spin-flip attempts/s per GPU",
        "value": attempts_per_step * args.steps / wall,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: 3D +-J EA L={L}, {R} realizations x {W} walkers, "
                               f"{S} multicanonical sweeps per step, checkerboard single-spin Metropolis",
                   "L": L, "realizations": R, "walkers_per_realization": W, "sweeps_per_step": S},
        "round_trips_per_s": trips / wall,
        "kernel_attempts_per_s": attempts_per_step * args.steps / (kernel_ms / 1e3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tops/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": f"k_muca_sweeps<{L}>", "avg_launch_ms": avg_launch_s * 1e3,
                     "alg_ops_per_attempt": ALG_OPS_PER_ATTEMPT},
    }
    b.close()
    if not args.no_cpu_baseline:
        b2, lnw2, klo2, ktop2 = setup(nfm, L, min(R, 8), W)
        line["cpu_baseline"] = cpu_baseline(b2, L, lnw2, klo2, ktop2)
        b2.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
