"""The round-trip-time comparison of Secs. III-V at test scale (L = 4, 64 realizations), end to end on
the GPU: weight iteration, the flat / 1/k / power-law production ensembles and parallel tempering
run until every realization has its round trips, then the host statistics of the library
(Frechet fits, quantile means, ratios with jackknife errors).

The parts are checked against the oracle elsewhere (sweeps, round-trip bookkeeping, recursion,
production weights, statistics); here: nothing is censored, the analysis agrees with the oracle's
statistics on the same times, and the paper's qualitative result at this size holds -- the
power-law ensemble needs fewer sweeps per round trip than the flat one (Table I: r = 1.6 at L = 4).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def campaign():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_08560_amd import campaign as c, nfm
    nfm.lib()
    return c


@pytest.fixture(scope="module")
def record(campaign):
    return campaign.compare(4, 64, min_trips=20, iter_sweeps=2000, n_max=40, chunk=1000, cap=400_000, first_id=300,
                            blocks=8, log=lambda s: print(s, flush=True))


def test_nothing_censored(record):
    assert all(v == 0 for v in record["censored"].values()), record["censored"]
    assert record["weight_iteration"]["converged"] == 64
    assert record["analysis"]["paired_realizations"] == 64


def test_analysis_matches_oracle(record):
    from oracle import stats as S
    tau = {m: np.array(t, float) for m, t in record["tau"].items()}
    for m, rec in record["analysis"]["methods"].items():
        print(m, {k: v for k, v in rec.items() if k != "r"}, rec.get("r"), flush=True)
        assert rec["tau_pop"] == pytest.approx(float(tau[m].mean()), rel=1e-12)
        (mu, beta, xi), f_orc = S.fit_ml(tau[m])
        f = rec["frechet"]
        got = (f["mu"], f["beta"], f["xi"])
        # the library's optimum, evaluated by the oracle, is at least as good as the oracle's; the
        # parameters agree where the likelihood is not flat in xi (xi -> 0 is the Gumbel limit)
        assert S.nll(got, tau[m]) <= f_orc + 1e-9 * abs(f_orc)
        if xi > 0.05:
            assert got == pytest.approx((mu, beta, xi), rel=1e-4)
        print(m, "oracle fit", (mu, beta, xi), flush=True)
        if m in ("flat", "invk"):
            want = S.relative_performance(tau[m], tau["pl"], eps=1e-4, method=0, blocks=8)
            print(m, "oracle r", want["r_pop"], want["r_eps"], flush=True)
            assert rec["r"]["r_pop"] == pytest.approx(want["r_pop"], rel=1e-12)
            assert rec["r"]["r_pop_err"] == pytest.approx(want["r_pop_err"], rel=1e-9)
            assert rec["r"]["r_eps"] == pytest.approx(want["r_eps"], rel=1e-4)
        elif m != "pl":
            # the population ratio and its jackknife error need no fits (blocks as in the oracle)
            n, k = len(tau[m]), 8
            full = tau[m].mean() / tau["pl"].mean()
            loo = []
            for j in range(k):
                keep = np.ones(n, bool)
                keep[j * n // k:(j + 1) * n // k] = False
                loo.append(tau[m][keep].mean() / tau["pl"][keep].mean())
            loo = np.array(loo)
            err = np.sqrt((k - 1) / k * np.sum((loo - loo.mean()) ** 2))
            assert rec["r"]["r_pop"] == pytest.approx(full, rel=1e-12)
            assert rec["r"]["r_pop_err"] == pytest.approx(err, rel=1e-9)


def test_power_law_beats_flat(record):
    r = record["analysis"]["methods"]["flat"]["r"]
    print(record["analysis"])
    assert r["r_pop"] > 1.0, r


def test_power_law_scan(campaign):
    rec = campaign.scan(4, 32, [1.0, 96.0], [-1.0, -3.6], min_trips=10, iter_sweeps=2000, n_max=40, chunk=1000,
                        cap=200_000, first_id=400, log=lambda s: print(s, flush=True))
    assert [(g["dE"], g["alpha"]) for g in rec["grid"]] == [(1.0, -1.0), (1.0, -3.6), (96.0, -1.0), (96.0, -3.6)]
    g = {(x["dE"], x["alpha"]): x for x in rec["grid"]}
    # the paper's setting and the mild exponents sample the whole range
    for key in ((1.0, -1.0), (96.0, -1.0), (96.0, -3.6)):
        assert g[key]["censored"] == 0 and g[key]["tau_pop"] > 0, rec
    # a steep power law pinned near the ground state (dE = 1) traps the walkers there: slower
    # than the paper's setting, or no round trips at all within the cap
    steep = g[(1.0, -3.6)]
    assert steep["censored"] > 0 or steep["tau_pop"] > g[(96.0, -3.6)]["tau_pop"], rec


def test_estimators_run(campaign):
    rec = campaign.estimators(4, 32, 2000, n_max=40, wl_sweeps=200, first_id=500, log=lambda s: print(s, flush=True))
    print(rec, flush=True)
    assert rec["recursion_sweeps"]["converged"] == 32, rec
    assert rec["wang_landau_sweeps"]["converged"] == 32, rec
    assert rec["paired"] == 32 and rec["wl_fewer"] + rec["wl_more"] <= 32


def test_estimators_with_seed_network(campaign):
    log = lambda s: print(s, flush=True)
    mlp, net = campaign.train_seed_network([4], 256, 2000, 0.5, 40, epochs=20, first_id=2000, log=log)
    rec = campaign.estimators(4, 32, 2000, n_max=40, wl_sweeps=200, first_id=500, mlp=mlp, log=log)
    print(rec, flush=True)
    # with the fallback to the plain start every realization converges; few need it, and the
    # seed saves sweeps for most
    assert rec["mlp_seeded_sweeps"]["converged"] == 32, rec
    assert rec["seed_fallback"] <= 3, rec
    assert rec["seeded_fewer"] > rec["seeded_more"], rec
    # the seeded arm pays for its canonical run
    assert rec["mlp_seeded_sweeps"]["median"] >= campaign.CANON_BURN + campaign.CANON_SWEEPS
