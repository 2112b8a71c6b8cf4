"""Pins for the oracle's Philox4x32-10 (random-number layout of the sampler).

The oracle's block function is checked against rocRAND's independent
implementation (called, not copied) and for uniformity / bit balance.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE_SRC = os.path.join(ROOT, "oracle", "rocrand_philox_probe.cpp")


def _probe_binary(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers or g++ not available")
    out = str(tmp_path_factory.mktemp("probe") / "philox_probe")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           PROBE_SRC, "-o", out])
    return out


def test_philox_matches_rocrand(orc, tmp_path_factory):
    exe = _probe_binary(tmp_path_factory)
    rng = np.random.default_rng(7)
    rows = rng.integers(0, 2 ** 32, size=(400, 6), dtype=np.uint64)
    rows[0] = 0
    rows[1] = 0xFFFFFFFF
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    res = subprocess.run([exe], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(v) for v in line.split()] for line in res.stdout.strip().splitlines()], np.uint64)
    assert ref.shape == (400, 4)
    for r, expect in zip(rows, ref):
        got = orc.philox(r[:4].astype(np.uint32), r[4:].astype(np.uint32))
        assert np.array_equal(got.astype(np.uint64), expect)


def test_philox_uniform_and_bit_balanced(orc):
    n = 20000
    words = np.empty((n, 4), np.uint32)
    for c in range(n):
        words[c] = orc.philox([c, 3, 11, orc.TAG_ACC], [0x1234, 0x5678])
    flat = words.reshape(-1).astype(np.uint64)
    # each bit is set with probability 1/2: 80000 draws, sigma ~ 141
    bits = np.array([((flat >> b) & 1).sum() for b in range(32)])
    assert np.all(np.abs(bits - flat.size / 2) < 6 * np.sqrt(flat.size / 4))
    # top byte histogram, chi-square with 255 dof
    hist = np.bincount((flat >> 24).astype(np.int64), minlength=256)
    exp = flat.size / 256
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert 160 < chi2 < 370
