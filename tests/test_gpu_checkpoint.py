"""Checkpoint and resume through the C ABI (nfm_checkpoint / nfm_restore).

A run interrupted by a checkpoint and resumed -- in a fresh context of the same batch
description, whose workspace sits at another address, or in the same context after it ran on --
must continue exactly as the uninterrupted run: the sweep counter travels with the state, so the
random words are the same. Compared bit for bit: spins, walker state (energies, minima, round-trip
counters and stamps), histograms, traces, the recursion's state and tables, the tempering slots,
exchange counters and temperatures. A checkpoint of another batch is refused.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DSEED, WSEED = 20110856, 0x5EED


@pytest.fixture(scope="module")
def nfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_08560_amd import nfm as m
    m.lib()
    return m


def _batch(nfm, Ls, seed=WSEED, trace=40):
    b = nfm.Batch(Ls, [64] * len(Ls), DSEED, seed, first_real_id=70, trace_capacity=trace)
    return b


def _state(b, Ls):
    out = {"spins": b.get_spins(0, b.n_walkers), "walkers": b.read_walkers(), "hist": b.read_histograms(),
           "trace": b.read_trace(), "sweeps": b.sweep_counter}
    for r in range(len(Ls)):
        st = b.rec_get_state(r)
        for k, v in st.items():
            out[f"rec{r}_{k}"] = v.tolist() if isinstance(v, np.void) else v.copy()
        out[f"thr{r}"] = b.get_thresholds(r)
    return out


def _equal(a, b):
    assert a.keys() == b.keys()
    for k in a:
        x, y = a[k], b[k]
        if isinstance(x, tuple):
            for u, v in zip(x, y):
                assert np.array_equal(np.asarray(u), np.asarray(v)), k
        else:
            assert np.array_equal(np.asarray(x), np.asarray(y)), k


def _continue_muca(b):
    b.run_sweeps(70)
    b.rec_update(0.5)
    b.run_sweeps(33)
    b.sync()


def test_resume_multicanonical(nfm):
    Ls = [4, 6, 4, 8]
    print("checkpoint: multicanonical Ls", Ls, flush=True)
    a = _batch(nfm, Ls)
    a.init_couplings()
    a.init_spins()
    a.compute_energies()
    a.rec_init(nfm.PROFILE_POWER, 96.0, -3.6)
    for _ in range(3):
        a.run_sweeps(50)
        a.rec_update(0.5)
    a.run_sweeps(17)                      # mid-round: the histogram holds counts
    blob = a.checkpoint()
    _continue_muca(a)
    want = _state(a, Ls)
    # a fresh context of the same description
    b = _batch(nfm, Ls)
    b.restore(blob)
    _continue_muca(b)
    _equal(_state(b, Ls), want)
    # the first context rewound
    a.restore(blob)
    _continue_muca(a)
    _equal(_state(a, Ls), want)
    a.close()
    b.close()


def test_resume_across_launch_forms(nfm):
    """A run under the split persistent launch, checkpointed mid-round and resumed under the
    per-size launches (and the reverse), continues exactly as the uninterrupted run: the launch
    form travels with the checkpoint but does not change results."""
    Ls = [4, 8, 6, 4, 8]
    print("checkpoint: across launch forms Ls", Ls, flush=True)
    for first, second in ((dict(schedule=2, sweeps_per_launch=16), dict(schedule=0, sweeps_per_launch=0)),
                          (dict(schedule=0, sweeps_per_launch=0), dict(schedule=2, sweeps_per_launch=9))):
        a = _batch(nfm, Ls)
        a.init_couplings()
        a.init_spins()
        a.compute_energies()
        a.rec_init(nfm.PROFILE_POWER, 96.0, -3.6)
        a.set_tuning(**first)
        a.run_sweeps(40)
        a.rec_update(0.5)
        a.run_sweeps(21)
        blob = a.checkpoint()
        _continue_muca(a)
        want = _state(a, Ls)
        b = _batch(nfm, Ls)
        b.restore(blob)
        assert b.get_tuning()["schedule"] == first["schedule"]
        b.set_tuning(**second)
        _continue_muca(b)
        _equal(_state(b, Ls), want)
        a.close()
        b.close()


def _continue_pt(b, M):
    b.pt_run_sweeps(41)
    b.sync()
    return {"slots": b.pt_slots(), "acc": b.pt_exchanges(M), "walkers": b.read_walkers(),
            "spins": b.get_spins(0, b.n_walkers), "trace": b.read_trace(), "T1": b.pt_temps(1, M),
            "sweeps": b.sweep_counter}


def test_resume_tempering(nfm):
    Ls, M = [4, 6], 12
    print("checkpoint: tempering Ls", Ls, "M", M, flush=True)
    a = _batch(nfm, Ls)
    a.init_couplings()
    a.init_spins()
    a.compute_energies()
    a.pt_init(0.3 * (3.2 / 0.3) ** (np.arange(M) / (M - 1)))
    a.pt_run_sweeps(20)
    a.pt_adapt(M, 0.4, 0.6)               # per-realization temperatures now differ from the ladder
    a.pt_run_sweeps(15)
    blob = a.checkpoint()
    want = _continue_pt(a, M)
    b = _batch(nfm, Ls)
    b.restore(blob)
    got = _continue_pt(b, M)
    _equal(got, want)
    a.close()
    b.close()


def test_restore_refuses_another_batch(nfm):
    a = _batch(nfm, [4, 4])
    a.init_couplings()
    blob = a.checkpoint()
    for other in (_batch(nfm, [4, 4], seed=WSEED + 1), _batch(nfm, [4, 6]), _batch(nfm, [4, 4], trace=0)):
        with pytest.raises(nfm.NfmError) as e:
            other.restore(blob)
        assert e.value.status == nfm.NFM_EINVAL
        other.close()
    with pytest.raises(nfm.NfmError) as e:
        a.restore(blob[:-1])
    assert e.value.status == nfm.NFM_ESIZE
    with pytest.raises(nfm.NfmError):
        a.restore(np.zeros(64, np.uint8))
    a.close()
