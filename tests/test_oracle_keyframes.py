"""Pins of the keyframe-schedule oracle (oracle/keyframes.py): the generator's known-answer
outputs, hand-derived time steps in the paper's Replica and ScanNet++ settings, the
iteration counts the text fixes, and the uniformity of the random keyframe draw."""
import os

import numpy as np
import pytest

from oracle import keyframes as K

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def test_splitmix64_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 7
    for seed, k, out in rows:
        assert K.splitmix64(int(seed), int(k)) == int(out)


def test_replica_setting_by_hand():
    # m = 5, n = 3 (two random keyframe iterations), keyframe threshold 50
    s = K.Schedule(5, 3, 50, seed=7)
    assert s.step(0, 100) == (True, [0] * 5)
    assert s.step(1, 10) == (False, [1, 1, 1, 0])          # a list of one keyframe
    assert s.step(2, 60) == (True, [2] * 5)
    kf, it = s.step(3, 50)                                  # 50 is not above the threshold
    assert not kf and it[:3] == [3, 3, 3] and sorted(it[3:]) == [0, 2]
    assert s.step(4, 51) == (True, [4] * 5)
    kf, it = s.step(5, 0)
    assert not kf and it[:3] == [5, 5, 5] and len(it) == 5 and set(it[3:]) <= {0, 2, 4}
    assert len(set(it[3:])) == 2
    assert it[3:] == K.shuffled([0, 2, 4], 7, 5)[:2]
    assert s.keyframes == [0, 2, 4]


def test_scannetpp_setting_stores_every_frame():
    # m = 10, n = 1 with nine random iterations; every frame joins the list
    s = K.Schedule(10, 1, 50, store_all=True, seed=3)
    counts = [200, 5, 7, 80, 0, 0, 0, 0, 0, 0, 0, 0, 3]
    for f, c in enumerate(counts):
        before = list(s.keyframes)
        kf, it = s.step(f, c)
        assert kf == (c > 50)
        if kf:
            assert it == [f] * 10
        else:
            assert it[0] == f and len(it) == 1 + min(9, len(before))
            assert f not in it[1:] and set(it[1:]) <= set(before) and len(set(it[1:])) == len(it) - 1
        assert s.keyframes == before + [f]


def test_negative_threshold_makes_every_frame_a_keyframe():
    s = K.Schedule(4, 2, -1)
    for f in range(5):
        assert s.step(f, 0) == (True, [f] * 4)
    assert s.keyframes == list(range(5))


def test_shuffle_is_a_permutation_that_depends_on_seed_and_frame():
    lst = list(range(100, 140))
    a, b, c = K.shuffled(lst, 1, 9), K.shuffled(lst, 2, 9), K.shuffled(lst, 1, 10)
    assert sorted(a) == lst and sorted(b) == lst and sorted(c) == lst
    assert a != b and a != c and a != lst
    assert K.shuffled(lst, 1, 9) == a                       # counter based: reproducible


@pytest.mark.parametrize("L,draw", [(7, 2), (12, 9)])
def test_random_keyframes_are_uniform(L, draw):
    # each keyframe of a list of L is drawn with probability draw / L; chi-square over
    # 4000 time steps (99.9% quantile of chi^2 with L - 1 degrees of freedom < 33)
    kfs = list(range(L))
    hits = np.zeros(L)
    T = 4000
    for f in range(T):
        for k in K.shuffled(kfs, 12345, f)[:draw]:
            hits[k] += 1
    expect = T * draw / L
    chi2 = ((hits - expect) ** 2 / expect).sum()
    assert chi2 < 33.0, (hits, chi2)
    # and the position of a keyframe in the shuffled list is uniform too
    first = np.zeros(L)
    for f in range(T):
        first[K.shuffled(kfs, 99, f)[0]] += 1
    chi2 = ((first - T / L) ** 2 / (T / L)).sum()
    assert chi2 < 33.0
