"""The library's keyframe schedule (gsr_schedule_*, host code) against the schedule oracle:
every time step's keyframe decision and iteration list must be identical.  Runs on the
CPU (no device work)."""
import numpy as np
import pytest

from oracle import keyframes as K
from paper_2408_12677_amd import _native as N
from paper_2408_12677_amd import rasterize as R


@pytest.mark.parametrize("m,n,thr,store_all,seed", [
    (5, 3, 50, False, 0),            # the paper's Replica setting
    (10, 1, 50, True, 12345),        # its ScanNet++ setting: every frame kept
    (4, 4, 10, False, 2 ** 64 - 1),  # no random iterations
    (6, 0, 100, True, 99),           # non-keyframes only replay keyframes
    (3, 1, -1, False, 7),            # every frame a keyframe
])
def test_schedule_matches_oracle(m, n, thr, store_all, seed):
    rng = np.random.default_rng(seed % 1000)
    ours, ref = R.Schedule(m, n, thr, store_all, seed), K.Schedule(m, n, thr, store_all, seed)
    # seeding counts: a burst at the start, then mostly few new Gaussians (revisits)
    counts = np.concatenate([rng.integers(100, 2000, 5), rng.geometric(0.05, 400) - 1])
    frame = 0
    for c in counts:
        frame += int(rng.integers(1, 3))             # frames need not be consecutive
        assert ours.step(frame, int(c)) == ref.step(frame, int(c)), (frame, c)
    assert ours.keyframes == ref.keyframes


def test_schedule_rejects_bad_arguments():
    import ctypes
    lib = N.load()
    h = ctypes.c_void_p()
    for m, n in ((2, 3), (1, -1)):
        s = N.ScheduleSettings(m, n, 50, 0, 0)
        assert lib.gsr_schedule_create(ctypes.byref(s), ctypes.byref(h)) == N.EINVAL
    sch = R.Schedule(5, 3)
    buf = (ctypes.c_int64 * 4)()
    cnt = ctypes.c_int32()
    assert lib.gsr_schedule_step(sch.h, 0, 10, buf, 4, ctypes.byref(cnt), None) == N.EINVAL   # cap < m
    assert lib.gsr_schedule_step(sch.h, -1, 10, buf, 5, ctypes.byref(cnt), None) == N.EINVAL
    assert sch.keyframes == []
