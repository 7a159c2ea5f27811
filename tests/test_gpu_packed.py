"""GPU parity of the packed path: two triplets per lane, one 16-bit half each.

The packed kernels keep every value as a biased positive integer below the
half-precision infinity pattern and take maxima with packed half-precision
instructions; the host admits a batch only when its scoring and lengths keep
every value in that range. Scores are integers, so the bar is equality with
the oracle (and with the int32 path) on every triplet.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2605_28400_amd as ts
from paper_2605_28400_amd import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PK_SHAPES = [((4, 4), 2), ((4, 4), 3), ((8, 4), 2), ((4, 8), 2)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run(torch, trips, sc=None, packed=0, engine=0, tile=(0, 0), wpe=0, use_graph=False, reps=1):
    lens, off, words = ts.pack_batch(trips)
    plan = ts.Plan(lens, off, sc=sc, engine=engine, tile=tile, waves_per_simd=wpe, use_graph=use_graph,
                   packed=packed)
    d_words = torch.from_numpy(words.view(np.int32)).cuda()
    outs = []
    for _ in range(reps):
        d_scores = torch.full((len(trips),), -7, dtype=torch.int32, device="cuda")
        plan.run(d_words, d_scores)
        torch.cuda.synchronize()
        outs.append(d_scores.cpu().numpy().copy())
    info = plan.info()
    plan.close()
    return outs, info


def oracle_scores(trips, sub=oracle.DEFAULT_SUB, gap=oracle.DEFAULT_GAP):
    return np.asarray(oracle.score_batch(trips, sub, gap), dtype=np.int64)


@pytest.mark.parametrize("seed,count,max_len", [(41, 57, 40), (42, 200, 120), (43, 33, 300), (44, 2, 5),
                                                (45, 3, 70)])
def test_packed_batches_equal_oracle(torch_cuda, seed, count, max_len):
    # Fuzz batches with empty, one-residue and skewed sequences; odd counts
    # pair the last triplet with itself.
    trips = synth.fuzz(seed=seed, count=count, max_len=max_len)
    want = oracle_scores(trips)
    say(f"packed fuzz seed={seed} n={count}")
    outs, info = run(torch_cuda, trips, reps=2)
    assert info["packed"] == 1
    for got in outs:
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, [(int(q), [s.size for s in trips[q]], int(got[q]), int(want[q])) for q in bad[:5]]


@pytest.mark.parametrize("tile,wpe", PK_SHAPES)
def test_packed_shapes_equal_oracle(torch_cuda, tile, wpe):
    trips = synth.fuzz(seed=47, count=120, max_len=150)
    want = oracle_scores(trips)
    say(f"packed tile={tile} wpe={wpe}")
    outs, info = run(torch_cuda, trips, packed=2, tile=tile, wpe=wpe)
    assert info["packed"] == 1 and (info["tile_rows"], info["tile_cols"]) == tile
    assert (outs[0] == want).all()


def test_packed_other_scorings(torch_cuda):
    # Any scoring whose terms sub - 2*gap are all >= 0 runs packed (a term of
    # exactly 0 included); one with a negative term runs in int32.
    rng = np.random.default_rng(5)
    trips = synth.fuzz(seed=46, count=90, max_len=80)
    for gap, packed in ((-3, 1), (-1, 1), (0, 0)):
        m = rng.integers(-2, 4, size=(4, 4))
        sub = np.triu(m) + np.triu(m, 1).T
        if gap == -1:
            sub[0, 0] = -2  # a term of exactly 0
        sc = ts.scoring(sub=sub.tolist(), gap=gap)
        want = oracle_scores(trips, sub.tolist(), gap)
        say(f"packed scoring gap={gap}")
        outs, info = run(torch_cuda, trips, sc=sc)
        assert info["packed"] == packed, (gap, sub - 2 * gap)
        assert (outs[0] == want).all()


def test_packed_batch_8192_matches_golden(torch_cuda):
    with open(os.path.join(GOLDEN, "batch_8192.json")) as f:
        g = json.load(f)
    w = synth.batch_8192()
    want = np.asarray(g["scores"])
    for use_graph in (False, True):
        say(f"packed batch 8192 graph={use_graph}")
        outs, info = run(torch_cuda, w.triplets, engine=-1, use_graph=use_graph, reps=2)
        assert info["packed"] == 1 and info["engine"] == 0
        for got in outs:
            bad = np.flatnonzero(got != want)
            assert bad.size == 0, bad[:10]


def test_packed_equals_int32_and_alone(torch_cuda):
    # The same batch through both lane forms, and each triplet alone (the
    # pairing depends on the batch, the scores must not).
    rng = np.random.default_rng(48)
    trips = [tuple(synth.uniform_seq(rng, int(m)) for m in rng.integers(20, 200, 3)) for _ in range(41)]
    pk, info_pk = run(torch_cuda, trips)
    i32, info_32 = run(torch_cuda, trips, packed=1)
    assert info_pk["packed"] == 1 and info_32["packed"] == 0
    assert (pk[0] == i32[0]).all()
    perm = rng.permutation(len(trips))
    shuffled, _ = run(torch_cuda, [trips[p] for p in perm])
    assert (shuffled[0] == pk[0][perm]).all()
    for q in range(0, len(trips), 8):
        assert ts.score(trips[q]) == pk[0][q]


def test_packed_range_limit_falls_back_to_int32(torch_cuda):
    # A large match score (term 14 per residue pair) and ~500-residue
    # sequences: the largest value a lane could hold would pass the 16-bit
    # half's range, so the batch runs in int32 lanes, with the oracle's
    # scores; the same scoring on short sequences runs packed.
    sub = [[10 if x == y else -1 for y in range(4)] for x in range(4)]
    sc = ts.scoring(sub=sub, gap=-2)
    rng = np.random.default_rng(49)
    long = [tuple(synth.uniform_seq(rng, n) for n in (500, 480, 510)),
            tuple(synth.uniform_seq(rng, n) for n in (30, 31, 29))]
    short = [tuple(synth.uniform_seq(rng, n) for n in (60, 50, 55)) for _ in range(5)]
    for trips, packed in ((long, 0), (short, 1)):
        say(f"packed range limit packed={packed}")
        outs, info = run(torch_cuda, trips, sc=sc)
        assert info["packed"] == packed
        assert (outs[0] == oracle_scores(trips, sub, -2)).all()
