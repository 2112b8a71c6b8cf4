"""Learned start of the weight iteration: data, training and the paired evaluation.

The weight iteration of Sec. II (Muller, Schnabel, Janke) starts from W = 1 and needs several
rounds before the walkers reach the lowest energies and the histogram flattens. Here a small
network guesses ln Omega(E) of a realization from its couplings and a short T = 2 canonical run;
the guess seeds the recursion as a prior on the DOS steps (nfm_rec_seed_grid), and the
recursion decides the final estimate. Every step runs in the library's kernels: the canonical run, the
features, the recursion, the targets, the network's training (FP32) and inference (BF16); torch
only holds device tensors and shuffles minibatches.

    python -m paper_2011_08560_amd.seeding --train-L 6 8 10 --train-real 16384 \
        --eval-L 10 --eval-real 2048

trains on realizations of the listed sizes (ids from 0), evaluates on fresh realizations (ids
from 10^6) with and without the seed under the same seeds, sweeps per round and flatness
tolerance, and prints one JSON line with the iterations to converge of both arms. With
--bench-net it only times the network's training steps and BF16 inference.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import nfm

DSEED, WSEED = 20110856, 0x0C5C5C5
EVAL_FIRST_ID = 1_000_000


def make_batch(Ls, walkers=64, first_real_id=0, disorder_seed=DSEED, walker_seed=WSEED):
    b = nfm.Batch(list(Ls), [walkers] * len(Ls), disorder_seed, walker_seed, first_real_id=first_real_id)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    return b


def canonical_features(b, T=2.0, burn=100, sweeps=1000):
    """Short canonical run at temperature T (burn-in, then the measured sweeps) and the model's
    inputs from the couplings and that run's histogram. The walkers are then drawn afresh (the
    same initial spins), so that the weight iteration starts as it would without the run: from
    random states, which are in equilibrium under its first weights (W = 1)."""
    b.set_canonical(T)
    b.run_sweeps(burn)
    b.reset_histograms()
    b.run_sweeps(sweeps)
    x = b.features()
    b.reset_histograms()
    b.init_spins()
    b.compute_energies()
    return x


def iterate(b, n_sweeps, f_tol=0.5, n_max=50, profile=(0, 1.0, 0.0), initialized=False, therm=0.1, log=None):
    """Weight iterations until every realization has converged once or n_max rounds: each round
    runs therm * n_sweeps sweeps under the new weights before its n_sweeps measured sweeps (the
    update reads the histogram as equilibrium data). Returns the round (1-based) at which each
    realization first converged; n_max + 1 = censored. log (optional) receives a line per round
    once a minute."""
    if not initialized:
        b.rec_init(*profile)
    first = np.full(b.n_real, n_max + 1, np.int64)
    n_therm = int(round(therm * n_sweeps))
    t_log = time.time()
    for it in range(1, n_max + 1):
        if n_therm:
            b.run_sweeps(n_therm)
            b.reset_histograms()
        b.run_sweeps(n_sweeps)
        info = b.rec_update(f_tol)
        newly = (info["converged"] == 1) & (first > n_max)
        first[newly] = it
        if log and time.time() - t_log > 60:
            t_log = time.time()
            log(f"weight iteration round {it}: {int((first <= n_max).sum())}/{b.n_real} converged")
        if (first <= n_max).all():
            break
    return first


def converged_targets(b, first, n_max):
    """Targets of the realizations that converged (the rest are masked out entirely)."""
    y, m = b.rec_targets()
    ok = np.asarray(first <= n_max)
    import torch
    m = m * torch.tensor(ok.astype(np.float32), device=m.device)[:, None]
    return y, m, ok


def feature_norm(x):
    """Per-input mean and spread of the training inputs (spread floored for constant inputs)."""
    mean = x.mean(dim=0)
    sd = x.std(dim=0).clamp_min(1e-3)
    return np.stack([mean.cpu().numpy(), sd.cpu().numpy()]).astype(np.float32)


def train(mlp, x, y, mask, epochs=50, batch=256, lr=1e-3, seed=0, val_frac=0.1, log=None):
    """Adam on the masked MSE, minibatches of `batch` realizations, a held-out fraction of
    realizations for the validation loss. Returns (train losses per epoch, validation loss)."""
    import torch
    n = x.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(n, generator=g)
    n_val = int(round(val_frac * n)) if n >= 20 else 0
    val, tr = perm[:n_val].to(x.device), perm[n_val:].to(x.device)
    mlp.set_params(norm=feature_norm(x[tr]))
    losses = []
    for ep in range(epochs):
        order = tr[torch.randperm(len(tr), generator=g).to(x.device)]
        tot, cnt = 0.0, 0
        for s in range(0, len(order), batch):
            idx = order[s:s + batch]
            if len(idx) == 0:
                continue
            xb, yb, mb = x[idx].contiguous(), y[idx].contiguous(), mask[idx].contiguous()
            mlp.train_step(xb, yb, mb, lr=lr)
            tot += mlp.last_loss() * len(idx)
            cnt += len(idx)
        losses.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4g}")
    val_loss = None
    if n_val:
        vals = []
        for s in range(0, n_val, batch):
            idx = val[s:s + batch]
            vals.append(mlp.loss_grad(x[idx].contiguous(), y[idx].contiguous(), mask[idx].contiguous()) * len(idx))
        val_loss = sum(vals) / n_val
    return losses, val_loss


def generate(Ls, n_per_L, n_sweeps, f_tol, n_max, chunk=4096, first_id=0, log=None):
    """Training data: per realization the model's inputs and the converged estimate's targets."""
    import torch
    xs, ys, ms = [], [], []
    stats = {}
    rid = first_id
    for L in Ls:
        done = 0
        conv = 0
        while done < n_per_L:
            n = min(chunk, n_per_L - done)
            b = make_batch([L] * n, first_real_id=rid)
            x = canonical_features(b)
            first = iterate(b, n_sweeps, f_tol, n_max, log=log)
            y, m, ok = converged_targets(b, first, n_max)
            xs.append(x)
            ys.append(y)
            ms.append(m)
            conv += int(ok.sum())
            b.close()
            done += n
            rid += n
        stats[L] = {"realizations": n_per_L, "converged": conv}
        if log:
            log(f"L={L}: {conv}/{n_per_L} converged within {n_max} rounds of {n_sweeps} sweeps")
    return torch.cat(xs), torch.cat(ys), torch.cat(ms), stats


def infer(mlp, x):
    """BF16 inference over any number of realizations, in chunks of the network's batch size."""
    import torch
    out = torch.empty((x.shape[0], nfm.Mlp.N_OUT), dtype=torch.float32, device=x.device)
    for s in range(0, x.shape[0], mlp.batch_max):
        mlp.infer_bf16(x[s:s + mlp.batch_max].contiguous(), out=out[s:s + mlp.batch_max])
    return out


CANON_SWEEPS = 100 + 1000   # the canonical run behind the features: burn-in and measured sweeps


def run_arm(mlp, L, n_real, n_sweeps, f_tol, n_max, first_id=EVAL_FIRST_ID, log=None):
    """One arm of the paired comparison on fresh realizations: the same seeds and the same
    canonical run for both; mlp = None runs the plain start, else the network's seed. Returns the
    round of first convergence per realization (n_max + 1 = censored), the seed's lowest level
    (-1 = plain start or rejected seed), the final lowest level k_lo and the final estimate as
    the training targets would see it (y = S/N on the 256-point grid and its mask)."""
    b = make_batch([L] * n_real, first_real_id=first_id)
    x = canonical_features(b)
    if mlp is None:
        k_seed = np.full(n_real, -1, np.int64)
        it = iterate(b, n_sweeps, f_tol, n_max, log=log)
    else:
        mlp.to_bf16()
        curves = infer(mlp, x)
        b.rec_init(0, 1.0, 0.0)
        k_seed = np.asarray(b.rec_seed_grid(curves), np.int64)
        it = iterate(b, n_sweeps, f_tol, n_max, initialized=True, log=log)
    info = b.rec_read_info()
    y, m = b.rec_targets()
    out = {"rounds": it, "k_seed": k_seed, "k_lo": np.asarray(info["k_lo"], np.int64),
           "y": y.cpu().numpy(), "mask": m.cpu().numpy()}
    b.close()
    return out


def evaluate(mlp, L, n_real, n_sweeps, f_tol, n_max, first_id=EVAL_FIRST_ID, log=None, full=False):
    """Paired comparison on fresh realizations: the same seeds, the same canonical run, then the
    plain start against the seeded one. Returns the rounds to converge of both arms (and, with
    full=True, both arms' records of run_arm)."""
    plain = run_arm(None, L, n_real, n_sweeps, f_tol, n_max, first_id, log)
    seeded = run_arm(mlp, L, n_real, n_sweeps, f_tol, n_max, first_id, log)
    if full:
        return plain, seeded
    return plain["rounds"], seeded["rounds"], seeded["k_seed"]


def bench_net(batch=256, steps=200, n_infer=16384, seed=7):
    """Throughput of the network's kernels on synthetic inputs (standard normal x, targets of
    spread 0.1, full masks): FP32 training steps (forward, back-propagation, Adam) on one
    minibatch of `batch` rows, and BF16 inference over n_infer rows in chunks of `batch`. A
    forward pass costs 2 x 75904 flops per row (81-128-128-128-256), a training step about three
    times that."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn(batch, nfm.Mlp.N_IN, generator=g).cuda()
    y = (0.1 * torch.randn(batch, nfm.Mlp.N_OUT, generator=g)).cuda()
    m = torch.ones(batch, nfm.Mlp.N_OUT).cuda()
    mlp = nfm.Mlp(batch_max=batch)
    mlp.init(seed)
    for _ in range(10):
        mlp.train_step(x, y, m, lr=1e-3)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        mlp.train_step(x, y, m, lr=1e-3)
    torch.cuda.synchronize()
    dt_train = (time.perf_counter() - t) / steps
    xi = torch.randn(n_infer, nfm.Mlp.N_IN, generator=g).cuda()
    mlp.to_bf16()
    infer(mlp, xi)
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = 20
    for _ in range(reps):
        infer(mlp, xi)
    torch.cuda.synchronize()
    dt_inf = (time.perf_counter() - t) / reps
    fwd = 2 * 75904
    return {"batch": batch, "train_step_us": dt_train * 1e6, "train_rows_per_s": batch / dt_train,
            "train_tflops": 3 * fwd * batch / dt_train / 1e12, "infer_rows": n_infer,
            "infer_us": dt_inf * 1e6, "infer_rows_per_s": n_infer / dt_inf,
            "infer_tflops": fwd * n_infer / dt_inf / 1e12, "final_loss": mlp.last_loss()}


def summary(it_plain, it_seed, k_seed, n_max):
    def arm(it):
        c = it > n_max
        return {"mean": float(it.mean()), "median": float(np.median(it)), "censored": int(c.sum())}
    return {"plain": arm(it_plain), "seeded": arm(it_seed), "seed_rejected": int((k_seed < 0).sum()),
            "fewer": int((it_seed < it_plain).sum()), "more": int((it_seed > it_plain).sum()),
            "paired_mean_gain": float((it_plain - it_seed).mean())}


def paired_report(plain, seeded, L, n_sweeps, n_max, therm=0.1):
    """The paired comparison at equal final flatness tolerance: rounds and total sweeps to the first
    converged round (a round is therm * n_sweeps thermalization plus n_sweeps measured sweeps; the
    seeded arm also pays the canonical run behind its features), censored counts, and whether the
    two arms reached the same estimate where both converged -- the same lowest level and the same
    S(E) within the estimates' noise (max |delta S| over the grid points both masks cover)."""
    N = L ** 3
    per_round = n_sweeps * (1.0 + therm)

    def arm(rec, extra):
        it = np.asarray(rec["rounds"])
        ok = it <= n_max
        tot = it * per_round + extra
        q = lambda v, p: float(np.quantile(v, p)) if len(v) else None
        return {"converged": int(ok.sum()), "censored": int((~ok).sum()),
                "rounds_median": q(it, 0.5), "rounds_p90": q(it, 0.9),
                "sweeps_median": q(tot, 0.5), "sweeps_p90": q(tot, 0.9),
                "rounds_median_converged": q(it[ok], 0.5)}
    itp, its = np.asarray(plain["rounds"]), np.asarray(seeded["rounds"])
    both = (itp <= n_max) & (its <= n_max)
    same_klo = plain["k_lo"][both] == seeded["k_lo"][both]
    dS = []
    for r in np.nonzero(both)[0]:
        cover = (plain["mask"][r] > 0) & (seeded["mask"][r] > 0)
        if cover.any():
            dS.append(float(np.abs(plain["y"][r][cover] - seeded["y"][r][cover]).max()) * N)
    dS = np.array(dS)
    return {"L": L, "realizations": int(len(itp)), "sweeps_per_round": n_sweeps, "n_max": n_max,
            "plain": arm(plain, 0.0), "seeded": arm(seeded, CANON_SWEEPS),
            "seed_rejected": int((np.asarray(seeded["k_seed"]) < 0).sum()),
            "fewer_rounds": int((its < itp).sum()), "more_rounds": int((its > itp).sum()),
            "both_converged": int(both.sum()),
            "same_lowest_level": int(same_klo.sum()),
            "seeded_lower_level": int((seeded["k_lo"][both] < plain["k_lo"][both]).sum()),
            "plain_lower_level": int((plain["k_lo"][both] < seeded["k_lo"][both]).sum()),
            "max_abs_dS_median": float(np.median(dS)) if len(dS) else None,
            "max_abs_dS_p90": float(np.quantile(dS, 0.9)) if len(dS) else None}


def _save(path, **arrays):
    np.savez(path, **{k: np.asarray(v) for k, v in arrays.items()})


def _load(path):
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-L", type=int, nargs="+", default=[6, 8, 10])
    ap.add_argument("--train-real", type=int, default=16384, help="training realizations in all")
    ap.add_argument("--eval-L", type=int, default=10)
    ap.add_argument("--eval-real", type=int, default=2048)
    ap.add_argument("--sweeps", type=int, default=10_000, help="sweeps per round of the weight iteration")
    ap.add_argument("--f-tol", type=float, default=0.5)
    ap.add_argument("--n-max", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--bench-net", action="store_true",
                    help="only time the network's training steps and BF16 inference on synthetic inputs")
    # the workflow in stages, so that a large run can be split over several processes
    ap.add_argument("--stage", choices=["data", "train", "eval", "report"],
                    help="data: training data of --train-L (ids from --first-id) into --out; train: the network "
                         "from --inputs data files into --out; eval: one arm (--arm) on --eval-real realizations "
                         "from --eval-first into --out (the seeded arm loads the network from --inputs); report: "
                         "the paired summary of --inputs plain and seeded arm files (no GPU)")
    ap.add_argument("--out")
    ap.add_argument("--inputs", nargs="*", default=[])
    ap.add_argument("--first-id", type=int, default=0)
    ap.add_argument("--arm", choices=["plain", "seeded"])
    ap.add_argument("--eval-first", type=int, default=EVAL_FIRST_ID)
    args = ap.parse_args(argv)
    if args.bench_net:
        print(json.dumps(bench_net(seed=args.seed)))
        return
    t0 = time.time()
    log = lambda s: print(f"[{time.time() - t0:7.1f}s] {s}", file=sys.stderr, flush=True)
    if args.stage == "data":
        per_L = int(math.ceil(args.train_real / len(args.train_L)))
        x, y, m, stats = generate(args.train_L, per_L, args.sweeps, args.f_tol, args.n_max, first_id=args.first_id,
                                  log=log)
        _save(args.out, x=x.cpu().numpy(), y=y.cpu().numpy(), m=m.cpu().numpy(),
              stats=json.dumps({str(k): v for k, v in stats.items()}))
        print(json.dumps({"stage": "data", "per_L": stats, "wall_s": time.time() - t0}))
        return
    if args.stage == "train":
        import torch
        parts = [_load(p) for p in args.inputs]
        x = torch.tensor(np.concatenate([p["x"] for p in parts]), device="cuda")
        y = torch.tensor(np.concatenate([p["y"] for p in parts]), device="cuda")
        m = torch.tensor(np.concatenate([p["m"] for p in parts]), device="cuda")
        mlp = nfm.Mlp(batch_max=256)
        mlp.init(args.seed)
        losses, val = train(mlp, x, y, m, epochs=args.epochs, lr=args.lr, seed=args.seed, log=log)
        params, norm = mlp.get_params()
        _save(args.out, params=params, norm=norm, losses=np.array(losses), val=np.float64(val if val else np.nan))
        print(json.dumps({"stage": "train", "rows": int(x.shape[0]), "rows_with_targets": int((m.sum(1) > 0).sum()),
                          "final_loss": losses[-1], "val_loss": val, "wall_s": time.time() - t0}))
        mlp.close()
        return
    if args.stage == "eval":
        mlp = None
        if args.arm == "seeded":
            net = _load(args.inputs[0])
            mlp = nfm.Mlp(batch_max=256)
            mlp.set_params(net["params"], net["norm"])
        rec = run_arm(mlp, args.eval_L, args.eval_real, args.sweeps, args.f_tol, args.n_max, args.eval_first, log)
        _save(args.out, arm=args.arm, first_id=np.int64(args.eval_first), **rec)
        it = rec["rounds"]
        print(json.dumps({"stage": "eval", "arm": args.arm, "realizations": args.eval_real,
                          "converged": int((it <= args.n_max).sum()), "rounds_median": float(np.median(it)),
                          "wall_s": time.time() - t0}))
        return
    if args.stage == "report":
        arms = {"plain": [], "seeded": []}
        for p in args.inputs:
            d = _load(p)
            arms[str(d.pop("arm"))].append(d)
        # chunks of realizations in id order; the two arms must cover the same ids
        ids = {a: [int(d["first_id"]) for d in sorted(ds, key=lambda d: int(d["first_id"]))] for a, ds in arms.items()}
        if ids["plain"] != ids["seeded"]:
            raise SystemExit(f"report: the arms cover different realizations: {ids}")
        cat = lambda ds: {k: np.concatenate([d[k] for d in sorted(ds, key=lambda d: int(d["first_id"]))])
                          for k in ds[0] if k != "first_id"}
        print(json.dumps(paired_report(cat(arms["plain"]), cat(arms["seeded"]), args.eval_L, args.sweeps,
                                       args.n_max)))
        return
    per_L = int(math.ceil(args.train_real / len(args.train_L)))
    x, y, m, stats = generate(args.train_L, per_L, args.sweeps, args.f_tol, args.n_max, log=log)
    mlp = nfm.Mlp(batch_max=256)
    mlp.init(args.seed)
    losses, val = train(mlp, x, y, m, epochs=args.epochs, lr=args.lr, seed=args.seed, log=log)
    it_p, it_s, ks = evaluate(mlp, args.eval_L, args.eval_real, args.sweeps, args.f_tol, args.n_max, log=log)
    out = {"train": {"L": args.train_L, "per_L": stats, "final_loss": losses[-1], "val_loss": val},
           "eval": {"L": args.eval_L, "realizations": args.eval_real,
                    **summary(it_p, it_s, ks, args.n_max)},
           "sweeps_per_round": args.sweeps, "f_tol": args.f_tol, "n_max": args.n_max,
           "wall_s": time.time() - t0}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
