"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Every test here runs on the CPU. Each pin would catch a different class of
plausible oracle bug: brute force catches anything; the closed forms and the
pairwise reductions catch wrong face/axis handling; symmetry catches an
index swapped between sequences; scaling catches a constant term.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2605_28400_amd import synth
from tests import pins

SUB = oracle.DEFAULT_SUB
GAP = oracle.DEFAULT_GAP
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def codes(s):
    return np.array(["ACGT".index(ch) for ch in s], dtype=np.uint8)


def test_delannoy_counts_of_enumerator():
    # Known 3-D Delannoy numbers: every alignment is enumerated exactly once.
    want = [1, 13, 409, 16081]
    for n, w in enumerate(want):
        seqs = [np.zeros(n, np.uint8)] * 3
        _, count = pins.enumerate_alignments(seqs, SUB, GAP)
        assert count == w == pins.delannoy3(n, n, n)
    assert pins.delannoy3(4, 4, 4) == 699121
    assert pins.delannoy3(4, 3, 3) == 50191


def test_nw_against_its_brute_force():
    rng = np.random.default_rng(11)
    for _ in range(60):
        s = synth.uniform_seq(rng, rng.integers(0, 6))
        t = synth.uniform_seq(rng, rng.integers(0, 6))
        sub = pins.random_symmetric_sub(rng)
        gap = int(rng.integers(-4, 2))
        assert pins.nw(s, t, sub, gap) == pins.nw_brute(s, t, sub, gap)


def test_hand_vectors():
    path = os.path.join(GOLDEN, "hand_vectors.txt")
    n = 0
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        *seqs, want = line.split()
        trip = [codes("" if s == "-" else s) for s in seqs]
        assert oracle.score(trip, SUB, GAP) == int(want), line
        n += 1
    assert n >= 10


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_small(seed):
    rng = np.random.default_rng(100 + seed)
    for trial in range(60):
        lens = rng.integers(0, 4, size=3)
        trip = [synth.uniform_seq(rng, int(n)) for n in lens]
        if trial % 2:
            sub, gap = pins.random_symmetric_sub(rng), int(rng.integers(-4, 2))
        else:
            sub, gap = SUB, GAP
        best, count = pins.enumerate_alignments(trip, sub, gap)
        assert count == pins.delannoy3(*map(int, lens))
        assert oracle.score(trip, sub, gap) == best, (lens, trip)


def test_brute_force_length_four():
    rng = np.random.default_rng(7)
    for lens in [(4, 3, 3), (4, 4, 2), (1, 4, 3)]:
        trip = [synth.uniform_seq(rng, n) for n in lens]
        sub = pins.random_symmetric_sub(rng)
        best, count = pins.enumerate_alignments(trip, sub, -2)
        assert count == pins.delannoy3(*lens)
        assert oracle.score(trip, sub, -2) == best


def test_asymmetric_scores_are_not_assumed_symmetric_in_brute_force():
    # A plain sanity check of the enumerator's column score on one column.
    col = (0, 1, pins.GAP)
    assert pins.column_sop(col, SUB, GAP) == -1 - 2 - 2


@pytest.mark.parametrize("seed", range(3))
def test_permutation_and_reversal_symmetry(seed):
    rng = np.random.default_rng(200 + seed)
    import itertools
    for _ in range(25):
        trip = [synth.uniform_seq(rng, int(n)) for n in rng.integers(0, 12, size=3)]
        sub = pins.random_symmetric_sub(rng)
        gap = int(rng.integers(-3, 1))
        ref = oracle.score(trip, sub, gap)
        for perm in itertools.permutations(range(3)):
            assert oracle.score([trip[p] for p in perm], sub, gap) == ref
        assert oracle.score([t[::-1] for t in trip], sub, gap) == ref


def test_identical_sequences_closed_form():
    rng = np.random.default_rng(5)
    for n in [0, 1, 2, 5, 17, 40]:
        x = synth.uniform_seq(rng, n)
        for match, mismatch, gap in [(1, -1, -2), (3, 0, -1), (2, -5, 0)]:
            sub = oracle.simple_sub(match, mismatch)
            assert oracle.score([x, x, x], sub, gap) == 3 * n * match


def test_one_empty_reduces_to_pairwise():
    rng = np.random.default_rng(6)
    empty = np.zeros(0, np.uint8)
    for _ in range(40):
        s = synth.uniform_seq(rng, rng.integers(0, 15))
        t = synth.uniform_seq(rng, rng.integers(0, 15))
        sub = pins.random_symmetric_sub(rng)
        gap = int(rng.integers(-4, 1))
        want = pins.nw(s, t, sub, gap) + gap * (len(s) + len(t))
        assert oracle.score([s, t, empty], sub, gap) == want
        assert oracle.score([empty, s, t], sub, gap) == want
        assert oracle.score([s, empty, t], sub, gap) == want


def test_two_empty_and_all_empty():
    empty = np.zeros(0, np.uint8)
    for n in [0, 1, 9, 33]:
        x = np.zeros(n, np.uint8)
        for gap in [-2, -1, 0, 3]:
            assert oracle.score([x, empty, empty], SUB, gap) == 2 * gap * n
            assert oracle.score([empty, empty, x], SUB, gap) == 2 * gap * n
    assert oracle.score([empty] * 3, SUB, GAP) == 0


def test_carrillo_lipman_bound_and_explicit_lower_bound():
    rng = np.random.default_rng(8)
    for _ in range(40):
        trip = [synth.uniform_seq(rng, int(n)) for n in rng.integers(0, 14, size=3)]
        sub = pins.random_symmetric_sub(rng)
        gap = int(rng.integers(-4, 1))
        s = oracle.score(trip, sub, gap)
        upper = (pins.nw(trip[0], trip[1], sub, gap) + pins.nw(trip[0], trip[2], sub, gap)
                 + pins.nw(trip[1], trip[2], sub, gap))
        assert s <= upper
        assert s >= pins.padded_alignment_score(trip, sub, gap)
    x = synth.uniform_seq(rng, 20)
    same = [x, x, x]
    assert oracle.score(same, SUB, GAP) == 3 * pins.nw(x, x, SUB, GAP)


def test_positive_scaling():
    rng = np.random.default_rng(9)
    for _ in range(20):
        trip = [synth.uniform_seq(rng, int(n)) for n in rng.integers(0, 12, size=3)]
        sub = pins.random_symmetric_sub(rng)
        gap = int(rng.integers(-4, 1))
        s = oracle.score(trip, sub, gap)
        for c in (2, 5):
            assert oracle.score(trip, sub * c, gap * c) == c * s


def test_batch_matches_single():
    rng = np.random.default_rng(10)
    trips = [[synth.uniform_seq(rng, int(n)) for n in rng.integers(0, 30, size=3)]
             for _ in range(50)]
    got = oracle.score_batch(trips, SUB, GAP, threads=4)
    assert [int(v) for v in got] == [oracle.score(t, SUB, GAP) for t in trips]
