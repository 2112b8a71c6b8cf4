"""Energy traces of a chosen range of walkers (nfm_trace_config) through the C ABI: the traced
rows equal the same walkers' rows of a trace of every walker, bit for bit, for multicanonical and
tempering sweeps; the range and its capacity survive a checkpoint; ranges outside the batch or
larger than the workspace's trace region are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DSEED, WSEED = 20110856, 0x7ACE
LS = [4, 6, 4]      # 192 walkers


@pytest.fixture(scope="module")
def nfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_08560_amd import nfm as m
    m.lib()
    return m


def _batch(nfm, cap=8):
    b = nfm.Batch(LS, [64] * len(LS), DSEED, WSEED, first_real_id=40, trace_capacity=cap)
    b.init_couplings()
    b.init_spins()
    b.compute_energies()
    b.set_canonical(2.5)
    return b


def test_range_rows_equal_the_full_trace(nfm):
    full = _batch(nfm)
    assert full.trace_range() == (0, 192, 8)
    full.run_sweeps(8)
    t1 = full.read_trace()
    full.reset_trace()
    full.run_sweeps(8)
    t2 = full.read_trace()
    assert t1.shape == t2.shape == (192, 8)
    part = _batch(nfm)
    part.trace_config(70, 40, 30)                  # 40 x 30 = 1200 <= 192 x 8 entries
    assert part.trace_range() == (70, 40, 30)
    part.run_sweeps(5)
    part.run_sweeps(11)                            # several calls
    tp = part.read_trace()
    assert tp.shape == (40, 16)
    assert np.array_equal(tp[:, :8], t1[70:110])
    assert np.array_equal(tp[:, 8:16], t2[70:110])
    # a checkpoint keeps the range, the capacity and the trace itself
    blob = part.checkpoint()
    other = _batch(nfm)
    other.restore(blob)
    assert other.trace_range() == (70, 40, 30)
    assert np.array_equal(other.read_trace(), tp)
    # no walkers traced at all
    part.trace_config(0, 0, 5)
    part.run_sweeps(2)
    assert part.read_trace().shape == (0, 0)
    for b in (full, part, other):
        b.close()


def test_range_under_tempering(nfm):
    M = 8
    temps = [0.5 * 1.3 ** m for m in range(M)]
    full = _batch(nfm)
    full.pt_init(temps)
    full.pt_run_sweeps(8)
    tf = full.read_trace()
    part = _batch(nfm)
    part.pt_init(temps)
    part.trace_config(100, 24, 8)
    part.pt_run_sweeps(8)
    assert np.array_equal(part.read_trace(), tf[100:124])
    full.close()
    part.close()


def test_bad_ranges_are_refused(nfm):
    b = _batch(nfm, cap=4)
    for args, status in (((-1, 5, 4), nfm.NFM_EINVAL), ((190, 3, 4), nfm.NFM_EINVAL), ((0, 10, -1), nfm.NFM_EINVAL),
                         ((0, 192, 5), nfm.NFM_ESIZE), ((0, 100, 8), nfm.NFM_ESIZE)):
        with pytest.raises(nfm.NfmError) as e:
            b.trace_config(*args)
        assert e.value.status == status, args
    assert b.trace_range() == (0, 192, 4)          # refused calls change nothing
    b.trace_config(0, 96, 8)                       # exactly the region
    b.close()
