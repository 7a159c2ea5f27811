"""Pins of the oracle's local variant (paper, Section II, "Local Alignments").

With v = 0 in every cell any cell can start an alignment (value 0) and any
cell can end one (the score is the largest value of the tensor), so the local
score is max(0, the best global score of any triple of contiguous substrings,
empty ones included). That is computed here from the brute-force enumerator
of explicit global alignments (tests/pins.py), with no dynamic programming
over the tensor, and compared with the oracle's recurrence.
"""
import numpy as np
import pytest

import oracle
from tests import pins


def substrings(s):
    out = {()}
    for i in range(len(s)):
        for j in range(i + 1, len(s) + 1):
            out.add(tuple(int(v) for v in s[i:j]))
    return sorted(out)


def local_brute(trip, sub, gap, memo):
    best = 0
    for a in substrings(trip[0]):
        for b in substrings(trip[1]):
            for c in substrings(trip[2]):
                key = (a, b, c, np.asarray(sub).tobytes(), gap)
                if key not in memo:
                    memo[key] = pins.enumerate_alignments([list(a), list(b), list(c)], sub, gap)[0]
                best = max(best, memo[key])
    return best


def local(trip, sub=oracle.DEFAULT_SUB, gap=oracle.DEFAULT_GAP):
    return oracle.score(trip, sub, gap, kind=oracle.LOCAL)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_local_equals_best_substring_alignment(seed):
    rng = np.random.default_rng(100 + seed)
    memo = {}
    subs = [oracle.DEFAULT_SUB, pins.random_symmetric_sub(rng, -3, 4)]
    for trial in range(24):
        lens = rng.integers(0, 3, size=3)
        if trial % 6 == 0:
            lens[trial % 3] = 3
        trip = [rng.integers(0, 4, size=int(n)).astype(np.uint8) for n in lens]
        sub = subs[trial % 2]
        gap = [-2, -1, -3][trial % 3]
        assert local(trip, sub, gap) == local_brute(trip, sub, gap, memo), (trip, gap)


def test_local_identical_sequences():
    rng = np.random.default_rng(7)
    for n in (1, 5, 9, 40):
        x = rng.integers(0, 4, size=n).astype(np.uint8)
        assert local([x, x, x]) == 3 * n  # every column: three matches of +1


def test_local_no_common_residue_is_zero():
    a = np.zeros(6, np.uint8)
    assert local([a, a + 1, a + 2]) == 0
    assert local([a, a + 1, a + 2], pins.random_symmetric_sub(np.random.default_rng(3), -5, -1)) == 0


def test_local_single_shared_residue():
    # One column of three equal residues scores 3 * match; nothing longer helps
    # when every other pairing mismatches and every gap costs.
    a = np.array([0, 1, 1], np.uint8)
    b = np.array([2, 0, 3], np.uint8)
    c = np.array([3, 3, 0], np.uint8)
    assert local([a, b, c]) == 3


def test_local_bounds_against_global():
    rng = np.random.default_rng(11)
    for _ in range(30):
        trip = [rng.integers(0, 4, size=int(n)).astype(np.uint8) for n in rng.integers(0, 25, 3)]
        lo = local(trip)
        assert lo >= 0 and lo >= oracle.score(trip)
        # Upper bound: a column gains at most 3 (three matching residues, the
        # one column kind that scores above 1), so the local score is at most
        # 3 * (the shortest length) plus the pairs of the two longer ones:
        # each column with two residues gains at most +1 - 2 - 2 < 0.
        assert lo <= 3 * min(len(s) for s in trip)


@pytest.mark.parametrize("seed", [5, 6])
def test_local_permutation_and_reversal_symmetry(seed):
    rng = np.random.default_rng(seed)
    sub = pins.random_symmetric_sub(rng, -3, 3)
    for _ in range(10):
        trip = [rng.integers(0, 4, size=int(n)).astype(np.uint8) for n in rng.integers(0, 18, 3)]
        want = local(trip, sub, -2)
        for p in ((1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0), (2, 0, 1)):
            assert local([trip[q] for q in p], sub, -2) == want
        assert local([s[::-1].copy() for s in trip], sub, -2) == want


def test_local_batch_matches_single():
    rng = np.random.default_rng(12)
    trips = [[rng.integers(0, 4, size=int(n)).astype(np.uint8) for n in rng.integers(0, 30, 3)]
             for _ in range(20)]
    got = oracle.score_batch(trips, kind=oracle.LOCAL, threads=4)
    assert [int(v) for v in got] == [local(t) for t in trips]
