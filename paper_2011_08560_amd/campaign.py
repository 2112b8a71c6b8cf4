"""Round-trip-time campaigns: the comparison of Secs. III-V and the power-law parameter scan.

For one lattice size, a batch of disorder realizations first runs the weight iteration (flat
target) to convergence; the converged estimate S = ln Omega then gives the production ensembles
of the methods compared in Table I -- flat (lnW = -S), 1/k (lnW = -ln sum_{E'<=E} Omega) and the
power law (lnW = -S + ln P_SH, Eq. (5)) -- and parallel tempering runs on the same realizations.
Each method runs until every realization has at least `min_trips` round trips between the lowest
energy found and the top (E >= 0; for tempering the mean energy of the hottest slot), in chunks,
realizations that are short of trips being run on ("requeued") up to a sweep cap, past which
they count as censored. The per-realization mean round-trip times then go through the host
statistics of the library: Frechet fits (Eq. (9)), shape xi, population and quantile means
(Eq. (14)), and the ratios r of Table I against the power law with jackknife errors. Every
simulation step runs in the library's kernels; this module only sequences calls.

    python -m paper_2011_08560_amd.campaign --L 4 --real 512 --min-trips 100
    python -m paper_2011_08560_amd.campaign --L 6 --real 256 --scan-dE 1 24 96 --scan-alpha -1 -2.4 -3.6
    python -m paper_2011_08560_amd.campaign --L 6 --real 256 --estimators

The second form is the scan of the power-law setting (Sec. II, Eq. (5)): the same realizations
and converged estimates, one production run per (dE, alpha). The third compares the estimators of
the density of states (the recursion of Sec. II and Wang-Landau) on sweeps to a flat histogram;
with --seed-train-L it also trains the seeding network on other realizations of those sizes and
adds the recursion seeded by its guess.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import nfm
from .seeding import canonical_features, generate, infer, iterate, make_batch, train

CANON_BURN, CANON_SWEEPS = 100, 1000   # the seeding network's canonical run (T = 2)

PT_TEMPS = [0.2 * 10.0 ** (m / 31.0) for m in range(32)]   # 32 temperatures geometric in [0.2, 2]
PL_PAPER = (96.0, -3.6)                                      # the paper's setting of Eq. (5)
METHODS = ("flat", "invk", "pl", "pt", "pt_adaptive")
# the paper's tempering protocol: M replicas per L, T_max > 3, temperatures adapted per realization
# for exchange rates in [0.4, 0.6]
PAPER_M = {3: 7, 4: 7, 5: 12, 6: 14, 8: 20}
ADAPT_T = (0.2, 3.2)


def converge(b, sweeps, f_tol, n_max, log=None):
    """Flat-target weight iteration until every realization converged once (or n_max rounds)."""
    first = iterate(b, sweeps, f_tol, n_max, profile=(nfm.PROFILE_FLAT, 1.0, 0.0), log=log)
    if log:
        log(f"weight iteration: {int((first <= n_max).sum())}/{len(first)} converged, "
            f"median round {float(np.median(first)):.0f}")
    return first


def run_until_trips(b, run, min_trips, chunk, cap, log=None, what=""):
    """Run `run(chunk)` until every realization has min_trips round trips or `cap` sweeps have
    run. Returns (tau per realization in sweeps, NaN = censored; sweeps run)."""
    done = 0
    t_log = time.time()
    while True:
        run(chunk)
        done += chunk
        tau, summ = b.rt_stats(min_trips=min_trips)
        if summ["n_censored"] == 0 or done >= cap:
            break
        if log and time.time() - t_log > 60:
            t_log = time.time()
            log(f"{what}: {done} sweeps so far, {int(summ['n_censored'])} realizations short of {min_trips} trips")
    if log:
        log(f"{what}: {done} sweeps, {int(summ['n_used'])} realizations with >= {min_trips} trips, "
            f"{int(summ['n_censored'])} censored")
    return tau, done


def production(b, method, min_trips, chunk, cap, pl=PL_PAPER, log=None):
    """Round-trip times of one multicanonical production ensemble."""
    prof = {"flat": (nfm.PROFILE_FLAT, 1.0, 0.0), "invk": (nfm.PROFILE_INVK, 1.0, 0.0),
            "pl": (nfm.PROFILE_POWER, pl[0], pl[1])}[method]
    b.rec_production(*prof)
    b.reset_round_trips()
    return run_until_trips(b, b.run_sweeps, min_trips, chunk, cap, log, method)


def adapt_temperatures(b, M, rounds=40, sweeps=500, band=(0.4, 0.6), log=None):
    """Equilibration with temperature adaptation per realization (nfm_pt_adapt) until every
    pair's exchange rate lies in the band or `rounds` are spent. Returns (rounds, last rates)."""
    rates = None
    for it in range(1, rounds + 1):
        b.pt_run_sweeps(sweeps)
        rates, n_out = b.pt_adapt(M, *band)
        if n_out == 0:
            break
    if log:
        log(f"pt adaptation: {it} rounds of {sweeps} sweeps, rates in [{rates.min():.3f}, {rates.max():.3f}]")
    return it, rates


def tempering(b, L, min_trips, chunk, cap, burn=1000, adaptive=False, log=None, adapt_M=None, adapt_T=None,
              adapt_rounds=40, adapt_sweeps=500):
    """Round-trip times of parallel tempering (in PT sweeps) between each realization's lowest
    energy found by the weight iteration and the mean energy of the hottest slot (averaged over
    the batch after a burn-in). adaptive: the paper's protocol (M from PAPER_M, temperatures in
    ADAPT_T adapted per realization; adapt_M / adapt_T override them) instead of the fixed
    32-temperature ladder."""
    info = b.rec_read_info()
    b.compute_energies()
    extra = {}
    if adaptive:
        M = adapt_M or PAPER_M.get(L, 20)
        t0, t1 = adapt_T or ADAPT_T
        b.pt_init([t0 * (t1 / t0) ** (s / (M - 1)) for s in range(M)])
        rounds, rates = adapt_temperatures(b, M, rounds=adapt_rounds, sweeps=adapt_sweeps, log=log)
        rates = np.asarray(rates).reshape(b.n_real, M - 1)
        in_band = ((rates >= 0.4) & (rates <= 0.6)).all(axis=1)
        q = np.quantile(rates, [0.05, 0.5, 0.95])
        extra = {"M": M, "T_range": [t0, t1], "adapt_rounds": rounds, "rates_min": float(rates.min()), "rates_max": float(rates.max()),
                 "rates_mean": float(rates.mean()), "rates_q05_q50_q95": [float(x) for x in q],
                 "realizations_in_band": int(in_band.sum())}
        if log:
            log(f"pt adaptation: {int(in_band.sum())}/{b.n_real} realizations with every rate in [0.4, 0.6]; "
                f"rate quantiles 5/50/95 % {q[0]:.3f}/{q[1]:.3f}/{q[2]:.3f}")
    else:
        M = len(PT_TEMPS)
        b.pt_init(PT_TEMPS)
    b.pt_run_sweeps(burn)
    ws = b.read_walkers()
    slots = b.pt_slots()
    e_hot = float(np.mean(ws["E"][slots == M - 1]))
    e_top = int(math.floor(e_hot))
    for r in range(b.n_real):
        e_bot = b.e_base(r) + 4 * int(info["k_lo"][r])
        b.set_rt_bounds(r, e_bot, max(e_top, e_bot + 4))
    b.reset_round_trips()
    tau, done = run_until_trips(b, b.pt_run_sweeps, min_trips, chunk, cap, log, "pt_adaptive" if adaptive else "pt")
    return tau, done, e_top, extra


RUNNING_MEAN_POINTS = (0.01, 0.03, 0.1, 0.3, 1.0)


def analyse(taus: dict, ref="pl", eps=1e-4, blocks=0):
    """Fits and ratios over the realizations uncensored under every method (paired): per method
    tau_pop, the ML fit of Eq. (9) with delete-a-block jackknife errors of its parameters (Fig. 4),
    the distance sup |F_n - F| between the empirical and the fitted CDF (Fig. 3), the running mean
    of Eq. (12) over the realizations in their order (Fig. 5; at fractions RUNNING_MEAN_POINTS of
    the sample and in full), the quantile and distribution means (Eqs. (11), (14)), and the ratios
    r of Table I against the reference method with their jackknife errors."""
    ok = np.ones(len(next(iter(taus.values()))), bool)
    for t in taus.values():
        ok &= np.isfinite(t) & (t > 0)
    out = {"paired_realizations": int(ok.sum()), "eps": eps, "methods": {}}
    for m, t in taus.items():
        tt = t[ok]
        rec = {"tau_pop": float(tt.mean()) if len(tt) else None}
        if len(tt) >= 1:
            run = nfm.running_mean(tt)
            rec["running_mean"] = {f"{f:g}": float(run[max(1, int(round(f * len(tt)))) - 1])
                                   for f in RUNNING_MEAN_POINTS}
            rec["running_mean_series"] = [float(x) for x in run]
        if len(tt) >= 3:
            B = blocks if blocks and len(tt) - (len(tt) + blocks - 1) // blocks >= 3 else 0
            fit, err, used = nfm.frechet_fit_jackknife(tt, 0, B)
            rec.update({"frechet": {"mu": fit[0], "beta": fit[1], "xi": fit[2]},
                        "frechet_err": {"mu": err[0], "beta": err[1], "xi": err[2], "blocks": used},
                        "ks_distance": nfm.frechet_ks(fit, tt),
                        "quantile_mean": nfm.frechet_quantile_mean(fit, eps),
                        "mean": nfm.frechet_mean(fit), "median": float(np.median(tt))})
            if m != ref and ref in taus:
                rec["r"] = nfm.relative_performance(tt, taus[ref][ok], eps=eps, method=0, blocks=blocks)
                rec["r"].pop("fit_m")
                rec["r"].pop("fit_ref")
        out["methods"][m] = rec
    return out


def compare(L, n_real, methods=METHODS, min_trips=100, iter_sweeps=None, f_tol=0.5, n_max=60, chunk=None,
            cap=None, first_id=0, eps=1e-4, blocks=0, log=None, adapt_M=None, adapt_T=None, adapt_rounds=40,
            adapt_sweeps=500):
    """The comparison of Secs. III-V at one L (round trips of every method, their distributions
    and Table I's ratios); returns a JSON-able record."""
    iter_sweeps = iter_sweeps or 1000 * L * L
    chunk = chunk or 50 * L ** 3
    cap = cap or 1000 * chunk
    b = make_batch([L] * n_real, first_real_id=first_id)
    first = converge(b, iter_sweeps, f_tol, n_max, log)
    taus, cost = {}, {}
    for m in methods:
        if m.startswith("pt"):
            continue
        taus[m], cost[m] = production(b, m, min_trips, chunk, cap, log=log)
    rec = {"L": L, "realizations": n_real, "min_trips": min_trips,
           "weight_iteration": {"sweeps_per_round": iter_sweeps, "f_tol": f_tol, "n_max": n_max,
                                "converged": int((first <= n_max).sum())}}
    for m in ("pt", "pt_adaptive"):
        if m in methods:
            taus[m], cost[m], e_top, extra = tempering(b, L, min_trips, chunk, cap, adaptive=(m == "pt_adaptive"),
                                                       log=log, adapt_M=adapt_M, adapt_T=adapt_T,
                                                       adapt_rounds=adapt_rounds, adapt_sweeps=adapt_sweeps)
            rec[m] = {"e_top": e_top, **extra}
            if m == "pt":
                rec[m]["temperatures"] = [PT_TEMPS[0], PT_TEMPS[-1], len(PT_TEMPS)]
    b.close()
    rec["sweeps_run"] = cost
    rec["censored"] = {m: int((~np.isfinite(t)).sum()) for m, t in taus.items()}
    rec["analysis"] = analyse(taus, eps=eps, blocks=blocks)
    rec["tau"] = {m: [None if not np.isfinite(x) else float(x) for x in t] for m, t in taus.items()}
    return rec


def scan(L, n_real, dEs, alphas, min_trips=100, iter_sweeps=None, f_tol=0.5, n_max=60, chunk=None, cap=None,
         first_id=0, log=None, eps=1e-4, blocks=0):
    """Population mean round-trip time of the power-law ensemble over a (dE, alpha) grid, and each
    grid point's ratios r (Table I's r_pop and r_eps, Sec. V) against the first grid point with
    alpha = 0 (the flat target; else the first grid point), over the realizations uncensored at
    both, with jackknife errors. The round-trip times are returned under "tau" as well."""
    iter_sweeps = iter_sweeps or 1000 * L * L
    chunk = chunk or 50 * L ** 3
    cap = cap or 1000 * chunk
    b = make_batch([L] * n_real, first_real_id=first_id)
    converge(b, iter_sweeps, f_tol, n_max, log)
    grid, taus = [], []
    for dE in dEs:
        for a in alphas:
            tau, done = production(b, "pl", min_trips, chunk, cap, pl=(dE, a), log=log)
            tau = np.asarray(tau, float)
            ok = np.isfinite(tau)
            grid.append({"dE": dE, "alpha": a, "tau_pop": float(tau[ok].mean()) if ok.any() else None,
                         "median": float(np.median(tau[ok])) if ok.any() else None,
                         "censored": int((~ok).sum()), "sweeps": done})
            taus.append(tau)
    b.close()
    ref = scan_ratios(grid, taus, eps, blocks)
    return {"L": L, "realizations": n_real, "min_trips": min_trips, "grid": grid,
            "reference": {"dE": grid[ref]["dE"], "alpha": grid[ref]["alpha"]},
            "tau": {f"dE{g['dE']:g}_a{g['alpha']:g}": t for g, t in zip(grid, taus)}}


def scan_ratios(grid, taus, eps=1e-4, blocks=0):
    """Adds to each grid point the number of realizations uncensored at it and at the reference
    (the first point with alpha = 0, else the first point) and, for the others, r_pop and r_eps
    against the reference over those realizations (Sec. V, Table I's ratios, jackknife errors).
    Returns the reference's index."""
    ref = next((i for i, g in enumerate(grid) if g["alpha"] == 0), 0)
    for i, g in enumerate(grid):
        both = np.isfinite(taus[i]) & np.isfinite(taus[ref]) & (taus[i] > 0) & (taus[ref] > 0)
        g["paired"] = int(both.sum())
        if i != ref and both.sum() >= 3:
            r = nfm.relative_performance(taus[i][both], taus[ref][both], eps=eps, method=0, blocks=blocks)
            g["r_vs_reference"] = {k: r[k] for k in ("r_pop", "r_pop_err", "r_eps", "r_eps_err", "blocks")}
    return ref


def estimators(L, n_real, sweeps, f_tol=0.5, n_max=60, wl_sweeps=None, wl_flat=0.8, wl_ln_f0=None, wl_final=None,
               wl_max_steps=2000, first_id=0, mlp=None, log=None):
    """Sweeps each estimator needs until its flat-target weights give a flat histogram (f_tol) on
    the same realizations: the recursion from W = 1, and Wang-Landau (steps of wl_sweeps, ln f
    from wl_ln_f0 halved at flatness wl_flat down to wl_final) handed to the recursion, which then
    runs its rounds until the same convergence test passes; with a trained seeding network `mlp`
    also the recursion seeded by its guess (its canonical run's sweeps counted). Rounds run 10 %
    extra thermalization sweeps, counted. Returns a JSON-able record with per-realization totals.

    The batched update adds ln f per counted visit but only after a whole step, so ln f0 is sized
    to raise a level by about one per step at an even spread over the 3N/2 + 1 levels (a first
    ln f of 1 per visit, as in one-walker Wang-Landau, lets ln g run far past its true range
    between updates and the stages stall); wl_final defaults to six halvings below it."""
    wl_sweeps = wl_sweeps or max(sweeps // 10, 1)
    N = L ** 3
    wl_ln_f0 = wl_ln_f0 or (3 * N // 2 + 1) / (64 * wl_sweeps)   # make_batch: 64 walkers each
    wl_final = wl_final or wl_ln_f0 / 64
    per_round = sweeps + int(round(0.1 * sweeps))
    b = make_batch([L] * n_real, first_real_id=first_id)
    first = iterate(b, sweeps, f_tol, n_max)
    b.close()
    plain = np.where(first <= n_max, first * per_round, np.nan).astype(float)
    if log:
        log(f"recursion: {int((first <= n_max).sum())}/{n_real} converged, median {np.nanmedian(plain):.0f} sweeps")
    b = make_batch([L] * n_real, first_real_id=first_id)
    b.wl_init(wl_ln_f0)
    done_at = np.full(n_real, -1, np.int64)
    t_log = time.time()
    for step in range(1, wl_max_steps + 1):
        b.run_sweeps(wl_sweeps)
        info = b.wl_update(wl_flat, wl_final)
        newly = (info["done"] == 1) & (done_at < 0)
        done_at[newly] = step
        if (done_at > 0).all():
            break
        if log and time.time() - t_log > 60:
            t_log = time.time()
            log(f"wang-landau step {step}: {int((done_at > 0).sum())}/{n_real} done, "
                f"median stage {float(np.median(info['stage'])):.0f}")
    b.wl_to_rec()
    after = iterate(b, sweeps, f_tol, n_max, initialized=True)
    b.close()
    wl_ok = (done_at > 0) & (after <= n_max)
    wl_total = np.where(wl_ok, done_at * wl_sweeps + after * per_round, np.nan).astype(float)
    if log:
        log(f"wang-landau: {int((done_at > 0).sum())}/{n_real} reached ln f < {wl_final}, "
            f"{int(wl_ok.sum())} converged after the hand-over, median {np.nanmedian(wl_total):.0f} sweeps")
    seeded, k_seed, fallback = None, None, None
    if mlp is not None:
        b = make_batch([L] * n_real, first_real_id=first_id)
        x = canonical_features(b, burn=CANON_BURN, sweeps=CANON_SWEEPS)
        mlp.to_bf16()
        curves = infer(mlp, x)
        b.rec_init(nfm.PROFILE_FLAT, 1.0, 0.0)
        k_seed = np.asarray(b.rec_seed_grid(curves))
        it = iterate(b, sweeps, f_tol, n_max, initialized=True, log=log)
        b.close()
        # a seeded start that has not converged by n_max rounds falls back to the plain start: its
        # cost is then the n_max rounds spent plus the plain arm's sweeps
        canon = CANON_BURN + CANON_SWEEPS
        fallback = it > n_max
        seeded = np.where(fallback, canon + n_max * per_round + plain, canon + it * per_round).astype(float)
        if log:
            log(f"seeded recursion: {int((~fallback).sum())}/{n_real} converged from the seed, "
                f"{int(fallback.sum())} fell back to the plain start, median {np.nanmedian(seeded):.0f} sweeps, "
                f"{int((k_seed < 0).sum())} seeds rejected")
    both = np.isfinite(plain) & np.isfinite(wl_total)

    def arm(x):
        f = x[np.isfinite(x)]
        return {"converged": int(len(f)), "median": float(np.median(f)) if len(f) else None,
                "mean": float(f.mean()) if len(f) else None}
    return {"L": L, "realizations": n_real, "sweeps_per_round": sweeps, "f_tol": f_tol, "n_max": n_max,
            "wl": {"sweeps_per_step": wl_sweeps, "flat": wl_flat, "ln_f0": wl_ln_f0, "ln_f_final": wl_final,
                   "median_stages_steps": float(np.median(done_at[done_at > 0])) if (done_at > 0).any() else None,
                   "rounds_after_handover_median": float(np.median(after[after <= n_max])) if (after <= n_max).any() else None},
            "recursion_sweeps": arm(plain), "wang_landau_sweeps": arm(wl_total),
            "paired": int(both.sum()), "wl_fewer": int((wl_total[both] < plain[both]).sum()),
            "wl_more": int((wl_total[both] > plain[both]).sum()),
            **({} if seeded is None else {
                "mlp_seeded_sweeps": arm(seeded), "seed_rejected": int((k_seed < 0).sum()),
                "seed_fallback": int(fallback.sum()),
                "seeded_fewer": int((seeded[np.isfinite(seeded) & np.isfinite(plain)]
                                     < plain[np.isfinite(seeded) & np.isfinite(plain)]).sum()),
                "seeded_more": int((seeded[np.isfinite(seeded) & np.isfinite(plain)]
                                    > plain[np.isfinite(seeded) & np.isfinite(plain)]).sum())})}


def train_seed_network(Ls, n_real, sweeps, f_tol, n_max, epochs=40, seed=7, first_id=0, log=None):
    """A seeding network trained on converged estimates of n_real realizations of the sizes Ls
    (ids from first_id on)."""
    per_L = int(math.ceil(n_real / len(Ls)))
    x, y, m, stats = generate(Ls, per_L, sweeps, f_tol, n_max, first_id=first_id, log=log)
    mlp = nfm.Mlp(batch_max=256)
    mlp.init(seed)
    losses, val = train(mlp, x, y, m, epochs=epochs, seed=seed)
    if log:
        log(f"seeding network: {len(Ls)} sizes, loss {losses[-1]:.4g}, validation {val}")
    return mlp, {"L": list(Ls), "per_L": stats, "final_loss": losses[-1], "val_loss": val}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, nargs="+", default=[4])
    ap.add_argument("--real", type=int, default=256)
    ap.add_argument("--methods", nargs="+", default=list(METHODS), choices=METHODS)
    ap.add_argument("--min-trips", type=int, default=100)
    ap.add_argument("--iter-sweeps", type=int, default=0)
    ap.add_argument("--f-tol", type=float, default=0.5)
    ap.add_argument("--n-max", type=int, default=60)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--cap", type=int, default=0)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--first-id", type=int, default=0)
    ap.add_argument("--scan-dE", type=float, nargs="*")
    ap.add_argument("--scan-alpha", type=float, nargs="*")
    ap.add_argument("--estimators", action="store_true",
                    help="compare the recursion with Wang-Landau on sweeps to a flat histogram")
    ap.add_argument("--seed-train-L", type=int, nargs="*",
                    help="with --estimators: also the recursion seeded by a network trained on these sizes")
    ap.add_argument("--seed-train-real", type=int, default=2048)
    ap.add_argument("--save-tau", help="comparison: write every method's per-realization times to this .npz")
    ap.add_argument("--adapt-M", type=int, default=0, help="pt_adaptive: replicas (default: the paper's M for L)")
    ap.add_argument("--adapt-T", type=float, nargs=2, metavar=("TMIN", "TMAX"),
                    help="pt_adaptive: temperature range (default [0.2, 3.2])")
    ap.add_argument("--adapt-rounds", type=int, default=40)
    ap.add_argument("--adapt-sweeps", type=int, default=500)
    ap.add_argument("--analyse", nargs="+", metavar="NPZ",
                    help="no simulation: pool the methods of earlier --save-tau files (same L, realizations "
                         "and seeds; a later file's method replaces an earlier one's) and analyse them")
    args = ap.parse_args(argv)
    t0 = time.time()
    log = lambda s: print(f"[{time.time() - t0:7.1f}s] {s}", file=sys.stderr, flush=True)
    if args.analyse:
        # files of one size pool their methods; files of several sizes give one analysis per size
        groups = {}
        for path in args.analyse:
            with np.load(path, allow_pickle=False) as z:
                L = int(z["L"]) if "L" in z.files else None
                g = groups.setdefault(L, {"sources": [], "taus": {}, "cap": {}})
                g["sources"].append(path)
                for k in z.files:
                    if k.startswith("tau_"):
                        g["taus"][k[4:]] = z[k]
                    elif k.startswith("sweeps_"):
                        g["cap"][k[7:]] = int(z[k])
        recs = {}
        for L, g in groups.items():
            recs[L] = {"sources": g["sources"], "sweeps_run": g["cap"],
                       "censored": {m: int((~np.isfinite(t)).sum()) for m, t in g["taus"].items()},
                       "analysis": analyse(g["taus"], eps=args.eps, blocks=args.blocks)}
        for L, r in sorted(recs.items(), key=lambda kv: (kv[0] is None, kv[0] or 0)):
            for m, a in r["analysis"]["methods"].items():
                if "frechet" not in a:
                    continue
                rr = a.get("r", {})
                print(f"L={L} {m:12s} xi = {a['frechet']['xi']:.3f} +- {a['frechet_err']['xi']:.3f}  "
                      f"KS = {a['ks_distance']:.3f}  tau_pop = {a['tau_pop']:.4g}  running mean at n/10, n: "
                      f"{a['running_mean']['0.1']:.4g}, {a['running_mean']['1']:.4g}"
                      + (f"  r_pop = {rr['r_pop']:.3f}({rr['r_pop_err']:.3f}) r_eps = {rr['r_eps']:.3f}"
                         f"({rr['r_eps_err']:.3f})" if rr else ""), file=sys.stderr, flush=True)
        if len(recs) == 1:
            out = next(iter(recs.values()))
        else:
            out = {"by_L": {str(L): r for L, r in recs.items()}}
        print(json.dumps(out), flush=True)
        return
    for L in args.L:
        if args.estimators:
            sw = args.iter_sweeps or 1000 * L * L
            mlp, net = None, None
            if args.seed_train_L:
                # training realizations from ids beyond the compared ones
                mlp, net = train_seed_network(args.seed_train_L, args.seed_train_real, sw, args.f_tol, args.n_max,
                                              first_id=args.first_id + args.real, log=log)
            rec = estimators(L, args.real, sw, args.f_tol, args.n_max, first_id=args.first_id, mlp=mlp, log=log)
            if net:
                rec["seed_network"] = net
        elif args.scan_dE and args.scan_alpha:
            rec = scan(L, args.real, args.scan_dE, args.scan_alpha, args.min_trips, args.iter_sweeps or None,
                       args.f_tol, args.n_max, args.chunk or None, args.cap or None, args.first_id, log,
                       eps=args.eps, blocks=args.blocks)
            tau = rec.pop("tau")
            if args.save_tau:
                np.savez(args.save_tau, **{f"tau_{k}": t for k, t in tau.items()}, L=np.int64(L))
        else:
            rec = compare(L, args.real, args.methods, args.min_trips, args.iter_sweeps or None, args.f_tol,
                          args.n_max, args.chunk or None, args.cap or None, args.first_id, args.eps, args.blocks, log,
                          adapt_M=args.adapt_M or None, adapt_T=tuple(args.adapt_T) if args.adapt_T else None,
                          adapt_rounds=args.adapt_rounds, adapt_sweeps=args.adapt_sweeps)
            tau = rec.pop("tau")
            if args.save_tau:
                np.savez(args.save_tau, **{f"tau_{m}": np.array([np.nan if x is None else x for x in t], float)
                                          for m, t in tau.items()},
                         **{f"sweeps_{m}": np.int64(v) for m, v in rec["sweeps_run"].items()}, L=np.int64(L))
        rec["wall_s"] = time.time() - t0
        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
