"""Pins of the oracle's semi-global variant (paper, Section II, "Semi-Global
Alignments").

The three axes hold 0 and v stays -infinity, so an alignment starts at an axis
cell (a prefix of at most one sequence is skipped at no cost) and ends on a
last slice (at least one sequence is used to its end; the rest of the other
two is dropped at no cost). The semi-global score is therefore the best
global score over those prefix/suffix choices. That is computed here from the
brute-force enumerator of explicit global alignments (tests/pins.py), with no
dynamic programming over the tensor, and compared with the oracle's
recurrence. Valid for gap <= 0: there a move along an axis never beats the
axis value 0, so "set to 0" and "start anywhere on an axis" agree.
"""
import itertools

import numpy as np
import pytest

import oracle
from tests import pins


def semi_brute(trip, sub, gap, memo):
    lens = [len(s) for s in trip]
    best = None
    starts = [(0, 0, 0)] + [tuple(p if q == s else 0 for q in range(3))
                            for s in range(3) for p in range(1, lens[s] + 1)]
    for st in starts:
        for end in itertools.product(*[range(st[s], lens[s] + 1) for s in range(3)]):
            if all(end[s] != lens[s] for s in range(3)):
                continue  # no sequence used to its end: not on a last slice
            parts = tuple(tuple(int(v) for v in trip[s][st[s]:end[s]]) for s in range(3))
            key = (parts, np.asarray(sub).tobytes(), gap)
            if key not in memo:
                memo[key] = pins.enumerate_alignments([list(p) for p in parts], sub, gap)[0]
            best = memo[key] if best is None else max(best, memo[key])
    return best


def semi(trip, sub=oracle.DEFAULT_SUB, gap=oracle.DEFAULT_GAP):
    return oracle.score(trip, sub, gap, kind=oracle.SEMI_GLOBAL)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_semiglobal_equals_best_prefix_suffix_choice(seed):
    rng = np.random.default_rng(300 + seed)
    memo = {}
    subs = [oracle.DEFAULT_SUB, pins.random_symmetric_sub(rng, -3, 4)]
    for trial in range(24):
        lens = rng.integers(0, 3, size=3)
        if trial % 6 == 0:
            lens[trial % 3] = 3
        trip = [rng.integers(0, 4, size=int(n)).astype(np.uint8) for n in lens]
        sub = subs[trial % 2]
        gap = [-2, -1, -3, 0][trial % 4]
        assert semi(trip, sub, gap) == semi_brute(trip, sub, gap, memo), (trip, gap)


def test_semiglobal_identical_sequences():
    rng = np.random.default_rng(8)
    for n in (1, 5, 9, 40):
        x = rng.integers(0, 4, size=n).astype(np.uint8)
        assert semi([x, x, x]) == 3 * n  # every column: three matches of +1


def test_semiglobal_motif_inside_longer_sequences():
    # A motif shared by all three sits at different offsets: the skipped
    # prefix of one sequence and the dropped suffixes cost nothing, but the
    # prefixes of the other two are still aligned, so only one offset is free.
    motif = np.array([0, 1, 2, 3, 3, 2, 1, 0], np.uint8)
    a = np.concatenate([np.array([1, 1, 1, 1], np.uint8), motif])
    assert semi([a, motif, motif]) == 3 * len(motif)
    # Dropping the tails of two sequences is free as well.
    b = np.concatenate([motif, np.array([2, 2, 2], np.uint8)])
    assert semi([motif, b, b]) == 3 * len(motif)


def test_semiglobal_faces_follow_their_recurrence():
    # S0 = S1 = AC, S2 = C. Only the axes are free: M[1][1][0] aligns A with A
    # against a gap, 1 - 2 - 2 = -3, so the triple match C/C/C that follows
    # reaches -3 + 3 = 0, the value of the axis cell (0, 0, 1), which already
    # lies on the last slice k = 1. Nothing scores above 0 (every other column
    # has a gap pair costing at least 3 more than it gains).
    ac, c = np.array([0, 1], np.uint8), np.array([1], np.uint8)
    assert semi([ac, ac, c]) == 0
    assert semi([ac, ac, c]) == semi_brute([ac, ac, c], oracle.DEFAULT_SUB, -2, {})


def test_semiglobal_answer_is_on_the_last_slices_only():
    # S0 = AG, S1 = AT, S2 = AC. The inner cell (1, 1, 1) holds 3 (A/A/A), but
    # every way on to a last slice costs it: G/T/C scores -3 and a column with
    # a gap scores at most 1 - 4. The axis cell (2, 0, 0) lies on the last
    # slice i = 2 with value 0, and nothing on a last slice does better.
    ag, at, ac = (np.array(v, np.uint8) for v in ([0, 2], [0, 3], [0, 1]))
    assert semi([ag, at, ac]) == 0
    assert semi([ag, at, ac]) == semi_brute([ag, at, ac], oracle.DEFAULT_SUB, -2, {})


def test_semiglobal_with_an_empty_sequence_is_best_face_cell():
    # With c = 0 every cell of the face k = 0 lies on the last slice k = c.
    rng = np.random.default_rng(9)
    for _ in range(10):
        x = rng.integers(0, 4, size=int(rng.integers(0, 9))).astype(np.uint8)
        y = rng.integers(0, 4, size=int(rng.integers(0, 9))).astype(np.uint8)
        e = np.zeros(0, np.uint8)
        # Columns (r, r', -) score sub - 4 <= -3 and (r, -, -) score -4 with the
        # default scoring, so nothing beats the axis value 0.
        assert semi([x, y, e]) == 0


def test_semiglobal_between_global_and_local():
    rng = np.random.default_rng(13)
    for _ in range(30):
        trip = [rng.integers(0, 4, size=int(n)).astype(np.uint8) for n in rng.integers(0, 25, 3)]
        s = semi(trip)
        assert oracle.score(trip) <= s <= oracle.score(trip, kind=oracle.LOCAL)


@pytest.mark.parametrize("seed", [5, 6])
def test_semiglobal_permutation_symmetry(seed):
    rng = np.random.default_rng(seed)
    sub = pins.random_symmetric_sub(rng, -3, 3)
    for _ in range(10):
        trip = [rng.integers(0, 4, size=int(n)).astype(np.uint8) for n in rng.integers(0, 18, 3)]
        want = semi(trip, sub, -2)
        for p in ((1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0), (2, 0, 1)):
            assert semi([trip[q] for q in p], sub, -2) == want


def test_semiglobal_batch_matches_single():
    rng = np.random.default_rng(14)
    trips = [[rng.integers(0, 4, size=int(n)).astype(np.uint8) for n in rng.integers(0, 30, 3)]
             for _ in range(20)]
    got = oracle.score_batch(trips, kind=oracle.SEMI_GLOBAL, threads=4)
    assert [int(v) for v in got] == [semi(t) for t in trips]
