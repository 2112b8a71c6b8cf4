"""Failure handling on the CPU: a sampling process killed between chunks and resumed from what it
saved (spins, walker state, sweep counter) continues exactly as the uninterrupted run. The random
words are counter-based (Philox keyed by seed, realization, walker; counter by sweep and site), so
the state and the absolute sweep counter are all that has to survive; the device checkpoint holds
the same (its GPU tests compare a resumed run with the uninterrupted one)."""
import os
import signal
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DSEED, WSEED, RID, L, W = 20110856, 0xC0FFEE, 11, 4, 6
N1, N2 = 7, 5

CHILD = r"""
import sys, numpy as np
sys.path.insert(0, {root!r})
from oracle import oracle as orc
sys.path.insert(0, {tests!r})
from test_oracle_resume import setup
rz, tab = setup(orc)
orc.sample(rz, *tab, {n1})
np.savez({path!r}, S=rz.S, w=rz.w, t=np.int64(rz.t))
print("saved", flush=True)
for _ in range(100000):        # the run goes on until the process is killed (bounded all the same)
    orc.sample(rz, *tab, 1)
"""


def setup(orc):
    rz = orc.make_realization(L, DSEED, RID, WSEED, W)
    K, eb = rz.K, rz.eb
    k_top = (-eb + 3) // 4
    k_lo = max(0, k_top - int(0.45 * L ** 3))
    lnw = -0.7 * (eb + 4 * np.arange(k_lo, k_top + 1, dtype=np.float64))
    thr, row0 = orc.build_thresholds(K, lnw, k_lo, k_top)
    return rz, (thr, row0, eb + 4 * k_lo, eb + 4 * k_top)


def test_killed_sampler_resumes_bit_for_bit(orc, tmp_path):
    path = str(tmp_path / "state.npz")
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), n1=N1, path=path)
    child = subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, text=True)
    try:
        line = child.stdout.readline()
        assert line.strip() == "saved", line
    finally:
        child.send_signal(signal.SIGKILL)
        child.wait(timeout=60)
    assert child.returncode == -signal.SIGKILL      # killed mid-run, not finished

    # resume in this process from the saved state
    rz, tab = setup(orc)
    with np.load(path, allow_pickle=False) as z:
        rz.S[...] = z["S"]
        rz.w[...] = z["w"]
        rz.t = int(z["t"])
    assert rz.t == N1
    H_resumed, _ = orc.sample(rz, *tab, N2)

    # the uninterrupted run
    ref, tab = setup(orc)
    orc.sample(ref, *tab, N1)
    H_ref, _ = orc.sample(ref, *tab, N2)

    assert np.array_equal(rz.S, ref.S)
    assert np.array_equal(rz.w, ref.w)
    assert rz.t == ref.t == N1 + N2
    assert np.array_equal(H_resumed, H_ref)
    # and the state did move (the comparison is not between two idle runs)
    fresh, _ = setup(orc)
    assert not np.array_equal(fresh.S, ref.S)


def test_resume_from_the_wrong_counter_differs(orc):
    """The counter matters: resuming the same state at another sweep counter gives other random
    words, so a checkpoint without its counter could not resume exactly."""
    a, tab = setup(orc)
    orc.sample(a, *tab, N1)
    b, _ = setup(orc)
    b.S[...] = a.S
    b.w[...] = a.w
    b.t = N1 + 1
    orc.sample(a, *tab, N2)
    orc.sample(b, *tab, N2)
    assert not np.array_equal(a.S, b.S)
