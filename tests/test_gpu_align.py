"""GPU traceback (`trioseq_align`) against the CPU oracle.

Several alignments can be optimal, so what is unique is compared and the rest
is checked for validity: the returned score equals the oracle's optimal global
score; the alignment's own sum-of-pairs score, recomputed column by column
here, equals it too; each row without its gaps is the input sequence; no
column is all gaps; the three rows have one length. Runs are deterministic.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2605_28400_amd as ts
from paper_2605_28400_amd import synth
from tests import pins

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LETTER = {c: q for q, c in enumerate("ACGT")}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def check_alignment(trip, rows, score, sub=oracle.DEFAULT_SUB, gap=oracle.DEFAULT_GAP, want=None):
    if want is None:
        want = oracle.score(trip, sub, gap)
    assert score == want, (score, want)
    assert len({len(r) for r in rows}) == 1
    for q in range(3):
        assert [LETTER[ch] for ch in rows[q] if ch != "-"] == [int(v) for v in trip[q]], q
    total = 0
    for col in zip(*rows):
        assert col != ("-", "-", "-")
        total += pins.column_sop(tuple(pins.GAP if ch == "-" else LETTER[ch] for ch in col), sub, gap)
    assert total == want, (total, want)


def test_small_fuzz(gpu):
    trips = synth.fuzz(seed=61, count=40, max_len=30)
    for q, t in enumerate(trips):
        say(f"align fuzz #{q} lens={[s.size for s in t]}")
        rows, score = ts.align(t)
        check_alignment(t, rows, score)


def test_related_triplets_several_levels(gpu):
    rng = np.random.default_rng(62)
    for n in (60, 150, 333):
        t = synth.mutated_triplet(rng, n, 0.1)
        say(f"align related lens={[s.size for s in t]}")
        rows, score = ts.align(t)
        check_alignment(t, rows, score)


def test_skewed_and_degenerate_shapes(gpu):
    rng = np.random.default_rng(63)
    shapes = [(0, 0, 0), (0, 0, 40), (0, 200, 3), (1, 300, 1), (250, 0, 90), (2, 2, 400),
              (120, 7, 130)]
    for n in shapes:
        t = tuple(synth.uniform_seq(rng, m) for m in n)
        say(f"align shape {n}")
        rows, score = ts.align(t)
        check_alignment(t, rows, score)
    x = synth.uniform_seq(rng, 200)
    rows, score = ts.align((x, x, x))
    assert score == 3 * 200 and "-" not in "".join(rows)


def test_random_scoring_schemes(gpu):
    rng = np.random.default_rng(64)
    for trial in range(4):
        sub = pins.random_symmetric_sub(rng, -4, 4)
        gap = int(rng.integers(-5, 1))
        sc = ts.scoring(sub=sub, gap=gap)
        t = synth.mutated_triplet(rng, int(rng.integers(20, 120)), 0.15)
        say(f"align scoring trial {trial} gap={gap}")
        rows, score = ts.align(t, sc)
        check_alignment(t, rows, score, sub, gap)


def test_deterministic(gpu):
    t = synth.mutated_triplet(np.random.default_rng(65), 180, 0.2)
    assert ts.align(t) == ts.align(t)


def test_single_1k_matches_golden(gpu):
    # Full size: 1024 x 1000 x 1048; the optimum is the stored oracle score.
    with open(os.path.join(GOLDEN, "single_1k.json")) as f:
        g = json.load(f)
    t = synth.single_1k().triplets[0]
    say("align single_1k")
    rows, score = ts.align(t)
    check_alignment(t, rows, score, want=int(g["scores"][0]))


def test_batch_equals_single_calls(gpu):
    # Fuzz shapes, related triplets and one large triplet in one batch: every
    # result valid and equal to the triplet aligned alone.
    rng = np.random.default_rng(66)
    trips = synth.fuzz(seed=66, count=30, max_len=40)
    trips += [synth.mutated_triplet(rng, int(n), 0.1) for n in (90, 260)]
    say(f"align batch n={len(trips)}")
    got = ts.align_batch(trips)
    want = oracle.score_batch(trips)
    for q, (t, (rows, score)) in enumerate(zip(trips, got)):
        check_alignment(t, rows, score, want=int(want[q]))
    for q in (0, 7, len(trips) - 2, len(trips) - 1):
        assert ts.align(trips[q]) == got[q]


def test_batch_of_length_8(gpu):
    # The traceback size the paper measures: many triplets of length 8.
    rng = np.random.default_rng(67)
    trips = [synth.mutated_triplet(rng, 8, 0.2, lens=(8, 8, 8)) for _ in range(3000)]
    say("align batch of 3000 x length 8")
    got = ts.align_batch(trips)
    want = oracle.score_batch(trips)
    for q in range(0, len(trips), 7):
        check_alignment(trips[q], got[q][0], got[q][1], want=int(want[q]))
    assert [s for _, s in got] == [int(v) for v in want]
