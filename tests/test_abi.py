"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
symbol declared in include/nfm.h, and validates batch descriptions."""
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "nfm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nfm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2011_08560_amd import nfm
    if not os.path.exists(nfm.LIB_PATH):
        pytest.fail("libnfm.so is not built: run __graft_entry__.build()")
    return nfm


def test_exports_every_declared_symbol(lib):
    L = lib.lib()
    names = _declared()
    assert len(names) >= 30
    for n in names:
        assert hasattr(L, n), n


def test_workspace_validation(lib):
    assert lib.workspace_bytes([8], [64]) > 0
    assert lib.workspace_bytes([4, 12, 6], [64, 128, 64], trace_capacity=10) > lib.workspace_bytes([4, 12, 6], [64, 128, 64])
    for Ls, Ws in (([3], [64]), ([14], [64]), ([8], [32]), ([8], [0]), ([0], [64]), ([], []), ([4, 6], [64])):
        with pytest.raises(lib.NfmError) as e:
            lib.workspace_bytes(Ls, Ws)
        assert e.value.status == lib.NFM_EINVAL


def test_coupling_word_format(lib, orc):
    for L in (2, 4, 6, 8):
        J = orc.couplings(L, 123, 4)
        w = lib.pack_couplings(J, L)
        assert w.size == 3 * ((L ** 3 + 31) // 32)
        assert (lib.unpack_couplings(w, L) == J).all()
        # bit i of plane d set <=> J = -1
        N = L ** 3
        for d, i in ((0, 0), (1, N - 1), (2, N // 2)):
            JW = (N + 31) // 32
            assert ((int(w[d * JW + i // 32]) >> (i % 32)) & 1) == (1 if J[d * N + i] < 0 else 0)


def test_device_tensor_checks_refuse_what_the_kernels_cannot_take(lib):
    """Every device array the binding hands to the library must be float32, row-major, of the
    exact shape the kernels assume and on the context's GPU; anything else is refused before
    the library is called (shown here with CPU and meta tensors: the checks run in that order)."""
    import torch
    dev = torch.device("cuda", 0)
    good_shape = (5, 81)
    for bad, what in ((torch.zeros(good_shape, dtype=torch.float64), "dtype"),
                      (torch.zeros((81, 5), dtype=torch.float32).t(), "contiguous"),
                      (torch.zeros((5, 80), dtype=torch.float32), "shape"),
                      (torch.zeros((4, 81), dtype=torch.float32), "shape"),
                      (torch.zeros(5 * 81, dtype=torch.float32), "shape"),
                      (torch.zeros(good_shape, dtype=torch.float32), "on cuda"),
                      (torch.zeros(good_shape, dtype=torch.float32, device="meta"), "on cuda"),
                      (np.zeros(good_shape, np.float32), "torch tensor")):
        with pytest.raises(ValueError) as e:
            lib.check_device_tensor(bad, dev, good_shape, "x")
        assert what.split()[0] in str(e.value) or "tensor" in str(e.value), (what, str(e.value))


def test_negative_sweep_counts_are_refused(lib):
    with pytest.raises(ValueError):
        lib._sweep_count(-1)
    assert lib._sweep_count(0) == 0 and lib._sweep_count(2 ** 40) == 2 ** 40
