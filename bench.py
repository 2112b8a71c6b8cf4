"""Benchmark of the multicanonical sampler on one MI355X.

Workload (default, the L = 6 configuration): 1024 disorder realizations of the 3D bimodal EA
spin glass, 64 walkers each, weight iteration towards the power-law target
H(E) ~ (E - E_min + 1)^(-a), a = 1 (Eq. (5) with dE = 1, alpha = -a; Sec. II of Muller,
Schnabel, Janke). One step is one pass of the hot path over the batch: S multicanonical sweeps
of every walker (per-attempt minimum and round-trip bookkeeping, per-sweep histograms), then
the device weight update (recursion, re-anchoring, flatness test, next weights and tables).
Disorder is synthetic and seeded (±1 couplings with p = 1/2, as in the paper's own samples).

Prints ONE JSON line: spin-flip attempts per second of the whole job, round trips per second,
weight-iteration progress, the roofline of the sweep kernel (integer VALU issue) and the CPU
oracle running the same iteration on a bounded sample.
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

# Algorithmic integer lane-operations per spin-flip attempt (the word-parallel sweep's floor):
# Philox4x32-10 share 10 (2.5 rounds x (2 wide products + 2 three-input xors)), neighbour
# count 1, table address 2, acceptance 2, spin/energy update 2, bookkeeping check 1.
ALG_OPS_PER_ATTEMPT = 18.0
# MI355X 32-bit vector ALU peak from its unit counts and clock: 256 CUs x 4 SIMD x 32 lanes x
# 2.4 GHz = 78.6 T lane-ops/s, the rate behind the published FP32 vector figure (157.3 TFLOP/s,
# an FMA counting two). Measured on the chip, simple integer ops reach about 20-23 lanes per
# clock per SIMD, 32x32-bit products 8-14, and a lone wave issues one instruction per ~4.7 cycles.
PEAK_LANE_OPS = 256 * 4 * 32 * 2.4e9

CONFIGS = {
    # name: (mix [(L, realizations)], walkers per realization, sweeps per step, description)
    "c2": ([(6, 1024)], 64, 100_000, "L=6, 1024 realizations, power-law target a=1 (dE=1), 1e5 sweeps per weight iteration"),
    "c3": ([(8, 4096)], 64, 10_000, "L=8, 4096 realizations, power-law target (dE=96, alpha=-3.6), 1e4 sweeps per step"),
    "c1": ([(4, 32)], 64, 10_000, "L=4, 32 realizations, flat target, 1e4 sweeps per weight iteration"),
    "c4": ([(4, 4096), (6, 2048), (8, 1024), (10, 512), (12, 256)], 64, 4_096,
           "mixed L=4/6/8/10/12 x 4096/2048/1024/512/256 realizations, power-law target, autotuned launch"),
    "c3pt": ([(8, 4096)], 64, 10_000, "L=8, 4096 realizations, parallel tempering with 32 temperatures "
                                      "geometric in [0.2, 2] (two sets of 32 per realization), exchanges every sweep"),
}
PROFILES = {"c2": (1, 1.0, -1.0), "c3": (1, 96.0, -3.6), "c1": (0, 1.0, 0.0), "c4": (1, 1.0, -1.0),
            "c3pt": None}
DSEED = 20110856


def setup(nfm, mix, W, profile):
    Ls = [L for L, R in mix for _ in range(R)]
    b = nfm.Batch(Ls, [W] * len(Ls), disorder_seed=DSEED, walker_seed=DSEED + 1, first_real_id=0)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    if profile is None:
        M = 32
        b.pt_init([0.2 * 10.0 ** (m / (M - 1)) for m in range(M)])
        for r, L in enumerate(Ls):        # a configuration at T = 2 sits near E/N = -1.4; ground states near -1.7
            b.set_rt_bounds(r, int(-1.66 * L ** 3), int(-1.40 * L ** 3))
    else:
        b.rec_init(*profile)
    return b, Ls


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweeps_L6_c2_traffic.txt")
SWEEP_SOURCE = os.path.join(ROOT, "paper_2011_08560_amd", "csrc", "sweep.hip")


def measured_traffic(config, sweeps_per_launch):
    """HBM bytes per launch of the sweep kernel from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, each scaled by the same counter's reading for a copy of known size), or None
    when there is none for this workload or the kernel source changed since it was taken."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
        digest = hashlib.sha256(open(SWEEP_SOURCE, "rb").read()).hexdigest()
        if kv.get("source_sha256") != digest or kv.get("config") != config:
            return None
        if int(kv.get("sweeps_per_launch", -1)) != sweeps_per_launch:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _oracle_iteration(args):
    L, rid, W, sweeps, profile = args
    from oracle import oracle as orc
    rz = orc.make_realization(L, DSEED, rid, DSEED + 1, W)
    st = orc.recursion_init(rz)
    t0 = time.perf_counter()
    orc.weight_iterations(rz, st, n_iter=1, n_sweeps=sweeps, profile=profile[0], pl_dE=profile[1],
                          pl_alpha=profile[2], stop=False)
    return W * sweeps * L ** 3, time.perf_counter() - t0


def cpu_baseline(L, W, profile, seconds_target=15.0):
    """The oracle as it stands: one weight iteration (weights, sweeps, update) per realization,
    one process per core over distinct realizations, on a bounded sample."""
    cores = max(1, min(16, os.cpu_count() or 1))
    n, dt = _oracle_iteration((L, 0, 4, 20, profile))          # rate probe, 4 walkers x 20 sweeps
    per_core = n / dt
    sweeps = max(10, int(seconds_target * per_core / (W * L ** 3)))
    tasks = [(L, rid, W, sweeps, profile) for rid in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_iteration, tasks)
    wall = time.perf_counter() - t0
    total = sum(r[0] for r in res)
    return {"value": total / wall, "unit": "attempts/s", "cores": cores, "kind": "oracle",
            "sample": f"L={L}: {cores} realizations x {W} walkers, one weight iteration of {sweeps} sweeps each "
                      f"({total:.3g} attempts in {wall:.1f} s wall, {cores} processes)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--sweeps", type=int, default=0, help="sweeps per step (default: the config's)")
    ap.add_argument("--walkers", type=int, default=0, help="walkers per realization (default: the config's)")
    ap.add_argument("--speculate", type=int, default=-1, choices=[-1, 0, 1],
                    help="speculative table lookups: -1 automatic, 0 off, 1 on")
    ap.add_argument("--ws", type=int, default=0, choices=[0, 1, 2],
                    help="generator wave beside each sampling wave: 0 automatic, 1 never, 2 always")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a reference dispatch of known traffic "
                         "for hardware-counter calibration); outside the timed region")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported here "
              f"(realizations are independent: one process per GPU would take a range of them)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2011_08560_amd import nfm

    if args.copy_mib:
        src = torch.ones(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    mix, W, S, desc = CONFIGS[args.config]
    S = args.sweeps or S
    W = args.walkers or W
    profile = PROFILES[args.config]
    pt = profile is None
    b, Ls = setup(nfm, mix, W, profile)
    L = max(Ls)
    R = len(Ls)
    tuned = None
    if args.config == "c4":
        b.run_sweeps(64)                  # one short round so that the tables have their working shape
        b.rec_update(0.5)
        tuned, _ = b.autotune(calib_sweeps=256)
    else:
        # 1000 sweeps per launch: the rounds of 1e4 / 1e5 sweeps split into equal launches
        b.set_tuning(speculate=args.speculate, sweeps_per_launch=min(1000, S), ws=args.ws)
    stream = torch.cuda.current_stream()
    attempts_per_step = W * S * sum(l ** 3 for l in Ls)
    tn = b.get_tuning()
    groups = 1 if len(mix) == 1 or (not pt and tn["schedule"] == 1) else len(mix)
    launches_per_step = math.ceil(S / tn["sweeps_per_launch"]) * groups

    def step():
        if pt:
            b.pt_run_sweeps(S)
        else:
            b.run_sweeps(S)

    def update():
        return None if pt else b.rec_update(0.5)

    for _ in range(args.warmup):
        step()
        update()
    torch.cuda.synchronize()
    trips0 = int(b.read_realizations()["rt_count"].sum())

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = None
    for k in range(args.steps):
        ev[k][0].record(stream)
        step()
        ev[k][1].record(stream)
        info = update()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    trips = int(b.read_realizations()["rt_count"].sum()) - trips0
    sweep_ms = sum(s.elapsed_time(e) for s, e in ev)
    avg_launch_s = sweep_ms / 1e3 / (args.steps * launches_per_step)
    attempts_per_launch = attempts_per_step / launches_per_step
    achieved = ALG_OPS_PER_ATTEMPT * attempts_per_launch / avg_launch_s / 1e12
    peak = PEAK_LANE_OPS / 1e12
    kernel = b.last_kernel()   # the form the library chose for the timed launches

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
        "config": {"workload": f"{args.config}: 3D +-J EA {desc}; one step = "
                               + ("PT sweeps" if pt else "sweeps + device weight update"),
                   "mix": [[l, r] for l, r in mix], "realizations": R, "walkers_per_realization": W,
                   "sweeps_per_step": S,
                   "profile": None if pt else {"kind": ["flat", "power", "invk"][profile[0]], "dE": profile[1],
                                               "alpha": profile[2]}},
        "round_trips_per_s": trips / wall,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tops/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(args.config, tn["sweeps_per_launch"]) if S % tn["sweeps_per_launch"] == 0
                     else None,
                     "kernel": kernel, "avg_launch_ms": avg_launch_s * 1e3,
                     "alg_ops_per_attempt": ALG_OPS_PER_ATTEMPT, "speculate": args.speculate, "ws": args.ws},
    }
    if info is not None:
        line["weight_iterations"] = {"done": int(info["iterations"].max()),
                                     "converged_fraction": float(info["converged"].mean()),
                                     "median_flatness": float(np.median(info["flatness"]))}
    if tuned is not None:
        line["tuning"] = tuned
    b.close()
    if not args.no_cpu_baseline and not pt and len(mix) == 1:
        line["cpu_baseline"] = cpu_baseline(L, W, profile)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
