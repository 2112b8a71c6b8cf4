"""Stuck-walker watch (nfm_stuck_walkers) through the C ABI: flags and count equal the definition
evaluated on the walkers' own round-trip state read back (age in whole sweeps since the last
completed round trip, or since the round-trip state was cleared), for windows from 0 to beyond
the run, before and after a clearing of the round-trip state, and after a checkpoint restore."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DSEED, WSEED = 20110856, 0x57AC
LS = [4, 6, 4, 2]


@pytest.fixture(scope="module")
def nfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_08560_amd import nfm as m
    m.lib()
    return m


def _batch(nfm):
    b = nfm.Batch(LS, [64] * len(LS), DSEED, WSEED, first_real_id=70)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    b.rec_init(nfm.PROFILE_FLAT)
    return b


def _expected(b, since, window):
    ws = b.read_walkers()
    now = b.sweep_counter
    flags = np.zeros(b.n_walkers, np.uint8)
    for r, L in enumerate(LS):
        N = L ** 3
        w0 = b.walker_offset(r)
        for w in range(w0, w0 + 64):
            last = int(ws["t_last"][w]) if ws["rt_count"][w] > 0 else since * N
            age = (now * N - last) // N if last < now * N else 0
            flags[w] = age >= window
    return flags


def _check(nfm, b, since, windows):
    import torch
    for window in windows:
        want = _expected(b, since, window)
        flags = torch.full((b.n_walkers,), 7, dtype=torch.uint8, device=b.device)
        n = b.stuck_walkers(window, flags)
        assert n == int(want.sum()), (window, n, int(want.sum()))
        assert np.array_equal(flags.cpu().numpy(), want), window
        assert b.stuck_walkers(window) == n            # without flags


def test_stuck_flags_follow_the_definition(nfm):
    b = _batch(nfm)
    b.run_sweeps(400)
    ws = b.read_walkers()
    assert (ws["rt_count"] > 0).any()
    _check(nfm, b, 0, [0, 1, 3, 20, 100, 399, 400, 401, 10 ** 12])
    assert b.stuck_walkers(0) == b.n_walkers
    assert b.stuck_walkers(401) == 0                    # nothing is older than the run
    # after clearing the round-trip state, walkers without a new trip count from the clearing
    b.reset_round_trips()
    b.run_sweeps(30)
    _check(nfm, b, 400, [0, 5, 29, 30, 31])
    assert b.stuck_walkers(31) == 0
    # the clearing's sweep is part of a checkpoint
    blob = b.checkpoint()
    c = _batch(nfm)
    c.restore(blob)
    for window in (5, 30):
        assert c.stuck_walkers(window) == b.stuck_walkers(window)
    c.close()
    b.close()


def test_stuck_walkers_refuses_bad_arguments(nfm):
    import torch
    b = _batch(nfm)
    with pytest.raises(ValueError):
        b.stuck_walkers(-1)
    with pytest.raises(ValueError):
        b.stuck_walkers(5, torch.zeros(b.n_walkers - 1, dtype=torch.uint8, device=b.device))
    with pytest.raises(ValueError):
        b.stuck_walkers(5, torch.zeros(b.n_walkers, dtype=torch.int32, device=b.device))
    b.close()
