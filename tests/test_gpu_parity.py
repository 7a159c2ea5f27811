"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle.

Scores are integers, so the bar is equality. Inputs are seeded; sizes span
several panels with ragged tails, the degenerate shapes (empty and length-1
sequences, all-equal and all-different residues), every tile shape and both
engines. Full-size workloads compare against oracle scores stored under
tests/golden/ (written by tests/golden/make_golden.py, which calls only the
oracle).
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
SHAPES = [(4, 4), (8, 4), (4, 8)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_plan(torch, trips, engine, tile=(0, 0), sc=None, use_graph=False, reps=1, grid=0):
    lens, off, words = ts.pack_batch(trips)
    plan = ts.Plan(lens, off, sc=sc, engine=engine, tile=tile, use_graph=use_graph, grid=grid)
    d_words = torch.from_numpy(words.view(np.int32)).cuda()
    outs = []
    for _ in range(reps):
        d_scores = torch.full((max(len(trips), 1),), -7, dtype=torch.int32, device="cuda")
        plan.run(d_words, d_scores)
        torch.cuda.synchronize()
        outs.append(d_scores.cpu().numpy()[:len(trips)].copy())
    info = plan.info()
    plan.close()
    return outs if reps > 1 else outs[0], info


def oracle_scores(trips, sub=oracle.DEFAULT_SUB, gap=oracle.DEFAULT_GAP):
    return np.asarray(oracle.score_batch(trips, sub, gap), dtype=np.int64)


def load_golden(name):
    with open(os.path.join(GOLDEN, f"{name}.json")) as f:
        return json.load(f)


def test_single_small_fuzz(torch_cuda):
    trips = synth.fuzz(seed=21, count=40, max_len=12)
    want = oracle_scores(trips)
    for q, t in enumerate(trips):
        say(f"single fuzz #{q} lens={[s.size for s in t]}")
        assert ts.score(t) == want[q], (q, [s.size for s in t])


@pytest.mark.parametrize("tile", SHAPES)
def test_batch_fuzz(torch_cuda, tile):
    trips = synth.fuzz(seed=22, count=120, max_len=90)
    want = oracle_scores(trips)
    say(f"batch fuzz tile={tile} n={len(trips)}")
    got, info = run_plan(torch_cuda, trips, engine=0, tile=tile)
    assert info["engine"] == 0
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, [(int(q), [s.size for s in trips[q]], int(got[q]), int(want[q])) for q in bad[:5]]


@pytest.mark.parametrize("tile", SHAPES)
def test_wide_multi_panel(torch_cuda, tile):
    rng = np.random.default_rng(23)
    shapes = [(150, 90, 201), (64, 64, 64), (1, 130, 77), (97, 1, 160), (0, 70, 140),
              (200, 33, 0), (129, 129, 129), (33, 257, 65)]
    for n in shapes:
        t = tuple(synth.uniform_seq(rng, m) for m in n)
        want = oracle.score(t)
        say(f"wide tile={tile} lens={n}")
        got, info = run_plan(torch_cuda, [t], engine=1, tile=tile)
        # A triplet that fits one panel is never split.
        assert info["engine"] == (1 if info["panels"] > 0 else 0)
        assert int(got[0]) == want, (n, int(got[0]), want, info)


def test_wide_with_few_wavefronts(torch_cuda):
    # More panel jobs than wavefronts: waves pop panels in dependency order.
    rng = np.random.default_rng(24)
    t = tuple(synth.uniform_seq(rng, m) for m in (120, 170, 190))
    want = oracle.score(t)
    for grid in (1, 3, 7):
        say(f"wide grid={grid}")
        got, info = run_plan(torch_cuda, [t], engine=1, grid=grid)
        assert info["grid"] == grid
        assert int(got[0]) == want


def test_random_scoring_schemes(torch_cuda):
    rng = np.random.default_rng(25)
    for trial in range(6):
        sub = pins.random_symmetric_sub(rng, -4, 4)
        gap = int(rng.integers(-6, 1))
        sc = ts.scoring(sub=sub, gap=gap)
        trips = [tuple(synth.uniform_seq(rng, int(m)) for m in rng.integers(0, 80, 3))
                 for _ in range(30)]
        want = oracle_scores(trips, sub, gap)
        say(f"scoring trial {trial} gap={gap}")
        got, _ = run_plan(torch_cuda, trips, engine=0, sc=sc)
        assert (got == want).all()
        got1, _ = run_plan(torch_cuda, trips[:1], engine=1, sc=sc)
        assert int(got1[0]) == want[0]


def test_identical_and_disjoint_residues(torch_cuda):
    trips = []
    for n in (1, 31, 32, 33, 100):
        x = np.full(n, 2, np.uint8)
        trips.append((x, x, x))
        trips.append((np.zeros(n, np.uint8), np.ones(n, np.uint8), np.full(n, 3, np.uint8)))
    want = oracle_scores(trips)
    got, _ = run_plan(torch_cuda, trips, engine=0)
    assert (got == want).all()
    for q in (4, 5, 8):
        assert ts.score(trips[q]) == want[q]


def test_single_128_matches_golden(torch_cuda):
    g = load_golden("single_128")
    w = synth.single_128()
    assert [[int(s.size) for s in t] for t in w.triplets] == g["lengths"]
    say("single 128^3")
    assert ts.score(w.triplets[0]) == g["scores"][0]
    got, _ = run_plan(torch_cuda, w.triplets, engine=0)
    assert int(got[0]) == g["scores"][0]
    # The default options (scored by halves at this length), as the benchmark
    # times them: graph replays.
    outs, info = run_plan(torch_cuda, w.triplets, engine=-1, use_graph=True, reps=3)
    assert info["engine"] == 1 and info["panels"] == 50
    assert all(int(o[0]) == g["scores"][0] for o in outs)


def test_single_1k_matches_golden(torch_cuda):
    g = load_golden("single_1k")
    w = synth.single_1k()
    assert [[int(s.size) for s in t] for t in w.triplets] == g["lengths"]
    for tile in SHAPES:
        say(f"single 1024x1000x1048 tile={tile}")
        got, _ = run_plan(torch_cuda, w.triplets, engine=1, tile=tile)
        assert int(got[0]) == g["scores"][0]


def test_single_1k_default_path_matches_golden(torch_cuda):
    # The launch configuration the benchmark times for a lone triplet: default
    # options (scored by halves), eager and graph replays, and the synchronous
    # call twice (the second call reuses the cached plan).
    g = load_golden("single_1k")
    w = synth.single_1k()
    say("single 1024x1000x1048 default options")
    got, info = run_plan(torch_cuda, w.triplets, engine=-1)
    assert info["engine"] == 1 and int(got[0]) == g["scores"][0]
    outs, _ = run_plan(torch_cuda, w.triplets, engine=-1, use_graph=True, reps=3)
    assert all(int(o[0]) == g["scores"][0] for o in outs)
    assert ts.score(w.triplets[0]) == g["scores"][0]
    assert ts.score(w.triplets[0]) == g["scores"][0]


def test_single_4k_matches_golden(torch_cuda):
    g = load_golden("single_4k")
    w = synth.single_4k()
    assert [[int(s.size) for s in t] for t in w.triplets] == g["lengths"]
    for engine in (-1, 1):
        say(f"single 4096x4000x4150 engine={engine}")
        got, _ = run_plan(torch_cuda, w.triplets, engine=engine)
        assert int(got[0]) == g["scores"][0]


def test_batch_8192_matches_golden(torch_cuda):
    g = load_golden("batch_8192")
    w = synth.batch_8192()
    assert [[int(s.size) for s in t] for t in w.triplets] == g["lengths"]
    want = np.asarray(g["scores"])
    for engine, tile, use_graph in ((0, (0, 0), False), (0, (0, 0), True), (-1, (0, 0), False),
                                    (-1, (8, 4), True), (-1, (4, 8), False)):
        say(f"batch 8192 engine={engine} tile={tile} graph={use_graph}")
        got, _ = run_plan(torch_cuda, w.triplets, engine=engine, tile=tile, use_graph=use_graph)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, bad[:10]


def test_graph_replays_match_eager(torch_cuda):
    torch = torch_cuda
    trips = synth.fuzz(seed=26, count=64, max_len=70)
    want = oracle_scores(trips)
    lens, off, words = ts.pack_batch(trips)
    plan = ts.Plan(lens, off, engine=0, use_graph=True)
    d_words = torch.from_numpy(words.view(np.int32)).cuda()
    d_scores = torch.zeros(len(trips), dtype=torch.int32, device="cuda")
    for rep in range(4):
        d_scores.fill_(-5)
        junk = torch.randn(256, 256, device="cuda") @ torch.randn(256, 256, device="cuda")
        plan.run(d_words, d_scores)
        torch.cuda.synchronize()
        say(f"graph replay {rep}")
        assert (d_scores.cpu().numpy() == want).all()
        del junk
    plan.close()


def test_alone_equals_in_batch_and_order_free(torch_cuda):
    rng = np.random.default_rng(27)
    trips = [tuple(synth.uniform_seq(rng, int(m)) for m in rng.integers(20, 140, 3)) for _ in range(24)]
    batch, _ = run_plan(torch_cuda, trips, engine=0)
    perm = rng.permutation(len(trips))
    shuffled, _ = run_plan(torch_cuda, [trips[p] for p in perm], engine=0)
    assert (shuffled == batch[perm]).all()
    for q in range(0, 24, 5):
        assert ts.score(trips[q]) == batch[q]
    assert (batch == oracle_scores(trips)).all()


def test_autotune_picks_a_parity_clean_config(torch_cuda):
    torch = torch_cuda
    trips = synth.fuzz(seed=28, count=300, max_len=120)
    want = oracle_scores(trips)
    lens, off, words = ts.pack_batch(trips)
    d_words = torch.from_numpy(words.view(np.int32)).cuda()
    say("autotune fuzz batch")
    r = ts.autotune(lens, off, d_words, reps=2)
    assert r["tried"] >= 2 and r["rejected"] == 0, r
    assert r["best_ms"] <= r["reference_ms"] + 1e-9
    # A plan made afterwards with default options uses the tuned shape.
    plan = ts.Plan(lens, off, engine=0)
    info = plan.info()
    if r["best"]["waves_per_simd"]:
        assert (info["tile_rows"], info["tile_cols"]) == (r["best"]["tile_rows"], r["best"]["tile_cols"])
    d_scores = torch.full((len(trips),), -7, dtype=torch.int32, device="cuda")
    plan.run(d_words, d_scores)
    torch.cuda.synchronize()
    plan.close()
    assert (d_scores.cpu().numpy() == want).all()


def test_score_batch_packed_device_buffers(torch_cuda):
    # One call on device-resident inputs; repeated calls reuse the layout, a
    # different batch replaces it, and a call on another stream waits for it.
    torch = torch_cuda
    rng = np.random.default_rng(29)
    trips = [tuple(synth.uniform_seq(rng, int(m)) for m in rng.integers(0, 150, 3)) for _ in range(40)]
    trips2 = trips[:7] + [synth.mutated_triplet(rng, 300, 0.1)]
    for batch in (trips, trips, trips2, trips):
        lens, off, words = ts.pack_batch(batch)
        d_words = torch.from_numpy(words.view(np.int32)).cuda()
        d_off = torch.from_numpy(np.asarray(off, dtype=np.uint64).view(np.int64)).cuda()
        d_len = torch.from_numpy(np.asarray(lens, dtype=np.uint32).view(np.int32)).cuda()
        d_scores = torch.full((len(batch),), -7, dtype=torch.int32, device="cuda")
        say(f"score_batch_packed n={len(batch)}")
        ts.score_batch_packed(d_words, d_off, d_len, d_scores, len(batch))
        torch.cuda.synchronize()
        assert (d_scores.cpu().numpy() == oracle_scores(batch)).all()
    s2 = torch.cuda.Stream()
    with torch.cuda.stream(s2):
        d_scores = torch.full((len(trips),), -7, dtype=torch.int32, device="cuda")
        lens, off, words = ts.pack_batch(trips)
        d_words = torch.from_numpy(words.view(np.int32)).cuda()
        d_off = torch.from_numpy(np.asarray(off, dtype=np.uint64).view(np.int64)).cuda()
        d_len = torch.from_numpy(np.asarray(lens, dtype=np.uint32).view(np.int32)).cuda()
        ts.score_batch_packed(d_words, d_off, d_len, d_scores, len(trips), stream=s2)
    torch.cuda.synchronize()
    assert (d_scores.cpu().numpy() == oracle_scores(trips)).all()


def test_lone_triplet_half_split(torch_cuda):
    # A lone global triplet under automatic options is scored by halves (its
    # longest sequence cut in two, the second half swept reversed, the two
    # last-slice planes met). Compared with the classic split engine and the
    # oracle on odd lengths, ties for the longest, empty and length-1
    # sequences, and graph replays.
    rng = np.random.default_rng(30)
    shapes = [(256, 40, 33), (257, 257, 100), (300, 0, 0), (0, 311, 7), (1, 1, 400), (290, 290, 290),
              (64, 333, 1), (513, 200, 150)]
    for q, n in enumerate(shapes):
        if q % 2:
            t = synth.mutated_triplet(rng, max(n), 0.1, lens=n)
        else:
            t = tuple(synth.uniform_seq(rng, m) for m in n)
        want = oracle.score(t)
        say(f"half split lens={n}")
        got_half, info = run_plan(torch_cuda, [t], engine=-1)
        got_classic, _ = run_plan(torch_cuda, [t], engine=1)
        assert int(got_half[0]) == int(got_classic[0]) == want, (n, int(got_half[0]), int(got_classic[0]), want)
        assert ts.score(t) == want
    t = synth.mutated_triplet(rng, 400, 0.05, lens=(400, 380, 390))
    outs, _ = run_plan(torch_cuda, [t], engine=-1, use_graph=True, reps=4)
    assert all(int(o[0]) == oracle.score(t) for o in outs)
