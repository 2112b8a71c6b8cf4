"""Benchmark of the multicanonical sampler on one MI355X.

Workload (default, the mixed-size batch): 4096 / 2048 / 1024 / 512 / 256 disorder realizations
of the 3D bimodal EA spin glass at L = 4 / 6 / 8 / 10 / 12 in one persistent launch whose
walker packing and sweep-chunk size the library's autotuner picks, 64 walkers each, weight
iteration towards the power-law target H(E) ~ (E - E_min + 1)^(-1) (Eq. (5) with dE = 1,
alpha = -1; Sec. II of Muller, Schnabel, Janke). One step is one pass of the hot path over the
batch: S multicanonical sweeps of every walker (per-attempt minimum and round-trip bookkeeping,
per-sweep histograms), then the device weight update (recursion, re-anchoring, flatness test,
next weights and tables). Disorder is synthetic and seeded (+-1 couplings with p = 1/2, as in
the paper's own samples). The other configurations (--config) are the single-size workloads.

Prints ONE JSON line: spin-flip attempts per second of the whole job, round trips per second,
weight iterations to first convergence, the roofline of the sweep kernel (integer VALU issue)
and the CPU oracle running the same iteration on a bounded sample.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic integer lane-operations per spin-flip attempt, counted for what the method must do
# per attempt with a per-site neighbour scan: a quarter of a Philox4x32-10 call (5 wide products
# and 10 xors), six bond tests (~10 bit operations), the threshold lookup with its compare and
# select, the conditional flip with the energy/level update (~4) and the minimum and round-trip
# tracking (~5): about 45.
ALG_OPS_PER_ATTEMPT = 45.0
# The floor of this library's word-parallel sweep (neighbour counts for a whole plane string at
# once): Philox share 10, neighbour count 1, table address 2, acceptance 2, update 2, bookkeeping 1.
DESIGN_OPS_PER_ATTEMPT = 18.0
# MI355X 32-bit vector ALU peak from its unit counts and clock: 256 CUs x 4 SIMD x 32 lanes x
# 2.4 GHz = 78.6 T lane-ops/s, the rate behind the published FP32 vector figure (157.3 TFLOP/s,
# an FMA counting two).
PEAK_LANE_OPS = 256 * 4 * 32 * 2.4e9

MIX_C4 = [(4, 4096), (6, 2048), (8, 1024), (10, 512), (12, 256)]
CONFIGS = {
    # name: (mix [(L, realizations)], walkers per realization, sweeps per step, description)
    "c4": (MIX_C4, 64, 10_000,
           "mixed L=4/6/8/10/12 x 4096/2048/1024/512/256 realizations in one autotuned persistent launch, "
           "power-law target a=1 (dE=1), 1e4 sweeps per weight iteration"),
    "c2": ([(6, 1024)], 64, 100_000, "L=6, 1024 realizations, power-law target a=1 (dE=1), 1e5 sweeps per weight iteration"),
    "c3": ([(8, 4096)], 64, 10_000, "L=8, 4096 realizations, power-law target (dE=96, alpha=-3.6), 1e4 sweeps per step"),
    "c1": ([(4, 32)], 64, 10_000, "L=4, 32 realizations, flat target, 1e4 sweeps per weight iteration"),
    "c3pt": ([(8, 4096)], 64, 10_000, "L=8, 4096 realizations, parallel tempering with 32 temperatures "
                                      "geometric in [0.2, 2] (two sets of 32 per realization), exchanges every sweep"),
}
PROFILES = {"c2": (1, 1.0, -1.0), "c3": (1, 96.0, -3.6), "c1": (0, 1.0, 0.0), "c4": (1, 1.0, -1.0),
            "c3pt": None}
PT_M, PT_TMIN, PT_TMAX = 32, 0.2, 2.0
DSEED = 20110856
F_TOL = 0.5
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2011_08560_amd", "csrc", f)
                  for f in ("sweep.hip", "kernels.hpp", "philox.hpp", "nfm_internal.hpp")]


def kernel_source_digest() -> str:
    """SHA-256 over the sweep kernel's sources (counter summaries are valid while it matches)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def pt_temps():
    return [PT_TMIN * (PT_TMAX / PT_TMIN) ** (m / (PT_M - 1)) for m in range(PT_M)]


def pt_bounds(L):
    # a configuration at T = 2 sits near E/N = -1.4; ground states near -1.7
    return int(-1.66 * L ** 3), int(-1.40 * L ** 3)


def setup(nfm, mix, W, profile):
    Ls = [L for L, R in mix for _ in range(R)]
    b = nfm.Batch(Ls, [W] * len(Ls), disorder_seed=DSEED, walker_seed=DSEED + 1, first_real_id=0)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    if profile is None:
        b.pt_init(pt_temps())
        for r, L in enumerate(Ls):
            b.set_rt_bounds(r, *pt_bounds(L))
    else:
        b.rec_init(*profile)
    return b, Ls


def counter_summary(config, kernel, sweeps_per_launch, key):
    """A figure from a committed rocprofv3 counter summary under profiles/ (lines 'key: value')
    for this workload, kernel form and launch size (sweeps_per_launch None: any launch size, for
    per-attempt figures), or None when there is none or the kernel's sources changed since the
    counters were taken."""
    digest = kernel_source_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        kv = {}
        try:
            for line in open(path):
                if line.startswith("#") or ":" not in line:
                    continue
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        except OSError:
            continue
        if (key in kv and kv.get("config") == config and kv.get("kernel") == kernel
                and kv.get("source_sha256") == digest
                and (sweeps_per_launch is None or kv.get("sweeps_per_launch") == str(sweeps_per_launch))):
            try:
                return float(kv[key])
            except ValueError:
                return None
    return None


# ------------------------------------------------------------------ the CPU oracle on a bounded sample

def _oracle_iteration(args):
    """One weight iteration (weights, sweeps, update) of one realization, in the oracle."""
    L, rid, W, sweeps, profile = args
    from oracle import oracle as orc
    rz = orc.make_realization(L, DSEED, rid, DSEED + 1, W)
    st = orc.recursion_init(rz)
    t0 = time.perf_counter()
    orc.weight_iterations(rz, st, n_iter=1, n_sweeps=sweeps, profile=profile[0], pl_dE=profile[1],
                          pl_alpha=profile[2], stop=False)
    return W * sweeps * L ** 3, time.perf_counter() - t0


def _oracle_pt(args):
    """PT sweeps of one set of M configurations of one realization, in the oracle."""
    L, rid, sweeps = args
    from oracle import oracle as orc
    T = orc.pt_temperatures(PT_M, PT_TMIN, PT_TMAX)
    metro = orc.pt_metro_table(T)
    swap = orc.pt_swap_table(T, 3 * L ** 3 // 2 + 1)
    ps = orc.make_pt_set(L, DSEED, rid, DSEED + 1, PT_M, 0)
    e_bot, e_top = pt_bounds(L)
    t0 = time.perf_counter()
    orc.pt_sweeps(ps, metro, swap, e_bot, e_top, sweeps)
    return PT_M * sweeps * L ** 3, time.perf_counter() - t0


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return model, os.cpu_count() or 1, avail, share


def cpu_baseline(mix, W, profile, seconds_target=15.0):
    """The oracle as it stands, one process per core over distinct realizations (cycling through
    the batch's lattice sizes), each running one weight iteration (multicanonical) or PT sweeps
    of one set (tempering) sized to about seconds_target, on a bounded sample of the workload."""
    model, nproc, avail, share = host_cpu()
    cores = max(1, min(avail, share) if share > 0 else avail)
    Ls = [L for L, _ in mix]
    pt = profile is None
    tasks = []
    for c in range(cores):
        L = Ls[c % len(Ls)]
        if pt:
            n, dt = _oracle_pt((L, c, 2))
            sweeps = max(2, int(seconds_target * n / dt / (PT_M * L ** 3)))
            tasks.append((L, c, sweeps))
        else:
            n, dt = _oracle_iteration((L, c, 4, 10, profile))        # rate probe: 4 walkers x 10 sweeps
            sweeps = max(10, int(seconds_target * n / dt / (W * L ** 3)))
            tasks.append((L, c, W, sweeps, profile))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_pt if pt else _oracle_iteration, tasks)
    wall = time.perf_counter() - t0
    total = sum(r[0] for r in res)
    per = ", ".join(f"L={t[0]}: {t[-1] if pt else t[3]} sweeps" for t in tasks[:len(Ls)])
    what = (f"one PT set of {PT_M} configurations per process" if pt
            else f"one weight iteration of {W} walkers per process")
    return {"value": total / wall, "unit": "attempts/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} processes over distinct realizations, L cycling through {Ls}, {what} "
                      f"({per}); {total:.3g} attempts in {wall:.1f} s wall; subset-measured",
            "nproc": nproc, "cpus_available": avail, "cpu_model": model,
            "cores_reason": "one process per core of the host's CPU share (OMP_NUM_THREADS)" if share > 0
            else "one process per available core"}


# ------------------------------------------------------------------ weight iterations to converge

def first_convergence_summary(first_conv, Ls, cap):
    """Iterations to the first converged update (Sec. II recursion: flat to f_tol with no new
    minimum) per lattice size: median, 90th percentile and the count still unconverged at the
    cap (censored; a median or percentile that falls among them is reported as '>cap')."""
    out = []
    Ls = np.asarray(Ls)
    for L in sorted(set(Ls.tolist())):
        it = first_conv[Ls == L]
        n = len(it)
        cens = int((it < 0).sum())
        srt = np.sort(np.where(it < 0, cap + 1, it))

        def q(p):
            v = int(srt[min(n - 1, int(math.ceil(p * n)) - 1)])
            return v if v <= cap else f">{cap}"
        out.append({"L": int(L), "realizations": n, "converged": n - cens, "censored": cens,
                    "median": q(0.5), "p90": q(0.9)})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c4", choices=sorted(CONFIGS))
    ap.add_argument("--sweeps", type=int, default=0, help="sweeps per step (default: the config's)")
    ap.add_argument("--walkers", type=int, default=0, help="walkers per realization (default: the config's)")
    ap.add_argument("--speculate", type=int, default=-1, choices=[-1, 0, 1],
                    help="single-size configs: speculative table lookups: -1 automatic, 0 off, 1 on")
    ap.add_argument("--ws", type=int, default=0, choices=[0, 1, 2],
                    help="single-size configs: generator wave beside each sampling wave: 0 automatic, 1 never, 2 always")
    ap.add_argument("--tuning", default="",
                    help="mixed configs: a fixed launch configuration 'schedule,sweeps_per_launch,waves_per_cu,speculate' "
                         "instead of the autotuner's pick (to profile one configuration)")
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
    R = len(Ls)
    tuned = None
    if len(mix) > 1 and not pt:
        b.run_sweeps(64)                  # one short round so that the tables have their working shape
        b.rec_update(F_TOL)
        if args.tuning:
            sch, spl, wpc, spec = (int(x) for x in args.tuning.split(","))
            b.set_tuning(schedule=sch, sweeps_per_launch=spl, waves_per_cu=wpc, speculate=spec)
            tuned = b.get_tuning()
        else:
            # calibration runs of 1024 sweeps per candidate: shorter ones rank the candidates less reliably
            tuned, _ = b.autotune(calib_sweeps=1024)
    else:
        # 1000 sweeps per launch: the rounds of 1e4 / 1e5 sweeps split into equal launches
        b.set_tuning(speculate=args.speculate, sweeps_per_launch=min(1000, S), ws=args.ws)
    stream = torch.cuda.current_stream()
    attempts_per_step = (PT_M * (64 // PT_M) * (W // 64) if pt else W) * S * sum(l ** 3 for l in Ls)
    tn = b.get_tuning()
    # launches per step: per-size launches run one per size; the persistent forms one per chunk
    # (the split form's two concurrent queues count as one launch: they share one fork and join)
    groups = 1 if len(mix) == 1 or (not pt and tn["schedule"] in (1, 2)) else len(mix)
    launches_per_step = math.ceil(S / tn["sweeps_per_launch"]) * groups

    def step():
        if pt:
            b.pt_run_sweeps(S)
        else:
            b.run_sweeps(S)

    first_conv = np.full(R, -1, np.int64)
    n_updates = [0]

    def update():
        if pt:
            return None
        info = b.rec_update(F_TOL)
        n_updates[0] += 1
        newly = (info["converged"] != 0) & (first_conv < 0)
        first_conv[newly] = n_updates[0]
        return info

    for _ in range(args.warmup):
        step()
        update()
    torch.cuda.synchronize()
    trips0 = int(b.read_realizations()["rt_count"].sum())

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        step()
        ev[k][1].record(stream)
        update()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    trips = int(b.read_realizations()["rt_count"].sum()) - trips0
    sweep_ms = sum(s.elapsed_time(e) for s, e in ev)
    avg_launch_s = sweep_ms / 1e3 / (args.steps * launches_per_step)
    attempts_per_launch = attempts_per_step / launches_per_step
    kernel_rate = attempts_per_launch / avg_launch_s           # attempts/s inside the sweep kernels
    achieved = ALG_OPS_PER_ATTEMPT * kernel_rate / 1e12
    peak = PEAK_LANE_OPS / 1e12
    kernel = b.last_kernel()   # the form the library chose for the timed launches
    spl = tn["sweeps_per_launch"]
    traffic = counter_summary(args.config, kernel, spl, "traffic_bytes_per_launch") if S % spl == 0 else None
    if traffic is None:
        # a summary that fitted per-launch traffic over two launch sizes serves any launch size
        fixed = counter_summary(args.config, kernel, None, "traffic_bytes_fixed_per_launch")
        per_sweep = counter_summary(args.config, kernel, None, "traffic_bytes_per_sweep")
        if fixed is not None and per_sweep is not None:
            traffic = fixed + per_sweep * S / launches_per_step
    # instructions per attempt do not depend on the launch size (counters of one launch size serve)
    valu = counter_summary(args.config, kernel, None, "valu_lane_instructions_per_attempt")

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
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": kernel, "avg_launch_ms": avg_launch_s * 1e3, "launches_per_step": launches_per_step,
                     "attempts_per_launch": attempts_per_launch,
                     "alg_ops_per_attempt": ALG_OPS_PER_ATTEMPT,
                     "frac_at_design_floor_18_ops": DESIGN_OPS_PER_ATTEMPT * kernel_rate / PEAK_LANE_OPS,
                     "valu_lane_instructions_per_attempt": valu,
                     "valu_issue_frac": None if valu is None else valu * kernel_rate / PEAK_LANE_OPS},
    }
    if not pt:
        line["weight_iterations"] = {
            "f_tol": F_TOL, "sweeps_per_iteration": S, "cap": n_updates[0],
            "to_first_convergence": first_convergence_summary(first_conv, Ls, n_updates[0])}
    if tuned is not None:
        line["tuning"] = tuned
    b.close()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(mix, W, profile)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
