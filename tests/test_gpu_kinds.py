"""GPU parity of the semi-global and local kinds (paper, Section II) against the
CPU oracle, through the C ABI.

Scores are integers, so the bar is equality. Each case runs both kinds on the
same seeded inputs: whole-triplet jobs (one wavefront per triplet), split
triplets (panel jobs whose bests are folded across wavefronts), mixed
batches, few wavefronts, repeated runs and graph replays of one plan (the
per-run reset of the fold), random scoring schemes, the degenerate shapes, and
the full-size workloads in the launch configuration the benchmark times.
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
KINDS = [("semi-global", ts.SEMI_GLOBAL, oracle.SEMI_GLOBAL), ("local", ts.LOCAL, oracle.LOCAL)]
KIND_IDS = [k[0] for k in KINDS]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_plan(torch, trips, sc, engine=-1, use_graph=False, reps=1, grid=0, tile=(0, 0)):
    lens, off, words = ts.pack_batch(trips)
    plan = ts.Plan(lens, off, sc=sc, engine=engine, use_graph=use_graph, grid=grid, tile=tile,
                   waves_per_simd=2 if tile != (0, 0) else 0)
    d_words = torch.from_numpy(words.view(np.int32)).cuda()
    outs = []
    for _ in range(reps):
        d_scores = torch.full((max(len(trips), 1),), -7, dtype=torch.int32, device="cuda")
        plan.run(d_words, d_scores)
        torch.cuda.synchronize()
        outs.append(d_scores.cpu().numpy()[:len(trips)].copy())
    info = plan.info()
    plan.close()
    return (outs if reps > 1 else outs[0]), info


def want_of(trips, okind, sub=oracle.DEFAULT_SUB, gap=oracle.DEFAULT_GAP):
    return np.asarray(oracle.score_batch(trips, sub, gap, kind=okind), dtype=np.int64)


def related(rng, count, lo, hi):
    """Mutated-ancestor triplets (large local and semi-global scores)."""
    return [synth.mutated_triplet(rng, int(rng.integers(lo, hi + 1)), float(rng.uniform(0.02, 0.3)))
            for _ in range(count)]


def report(trips, got, want):
    bad = np.flatnonzero(got != want)
    return [(int(q), [s.size for s in trips[q]], int(got[q]), int(want[q])) for q in bad[:5]]


@pytest.mark.parametrize("name,kind,okind", KINDS, ids=KIND_IDS)
def test_single_small_fuzz(torch_cuda, name, kind, okind):
    trips = synth.fuzz(seed=41, count=30, max_len=12)
    want = want_of(trips, okind)
    sc = ts.scoring(kind=kind)
    for q, t in enumerate(trips):
        say(f"{name} single fuzz #{q} lens={[s.size for s in t]}")
        assert ts.score(t, sc) == want[q], (q, [s.size for s in t])


@pytest.mark.parametrize("tile", [(4, 4), (8, 4)], ids=["4x4", "8x4"])
@pytest.mark.parametrize("name,kind,okind", KINDS, ids=KIND_IDS)
def test_batch_whole_triplets(torch_cuda, name, kind, okind, tile):
    rng = np.random.default_rng(42)
    trips = synth.fuzz(seed=42, count=60, max_len=90) + related(rng, 60, 1, 120)
    want = want_of(trips, okind)
    say(f"{name} batch whole n={len(trips)} tile={tile}")
    got, info = run_plan(torch_cuda, trips, ts.scoring(kind=kind), engine=0, tile=tile)
    assert info["engine"] == 0 and (info["tile_rows"], info["tile_cols"]) == tile
    assert (got == want).all(), report(trips, got, want)
    # Split and mixed plans of the same tile shape.
    got1, info1 = run_plan(torch_cuda, related(rng, 1, 200, 200) + trips[:20], ts.scoring(kind=kind),
                           tile=tile)
    assert info1["engine"] == 2
    assert (got1[1:] == want[:20]).all()


@pytest.mark.parametrize("name,kind,okind", KINDS, ids=KIND_IDS)
def test_split_triplets(torch_cuda, name, kind, okind):
    rng = np.random.default_rng(43)
    shapes = [(150, 90, 201), (64, 64, 64), (1, 130, 77), (97, 1, 160), (0, 70, 140),
              (200, 33, 0), (129, 129, 129), (33, 257, 65), (65, 65, 300)]
    sc = ts.scoring(kind=kind)
    for q, n in enumerate(shapes):
        if q % 2:
            anc = synth.uniform_seq(rng, max(n))
            t = tuple(synth.fix_length(rng, synth.mutate(rng, anc, 0.1), m) for m in n)
        else:
            t = tuple(synth.uniform_seq(rng, m) for m in n)
        want = oracle.score(t, kind=okind)
        say(f"{name} split lens={n}")
        got, info = run_plan(torch_cuda, [t], sc, engine=1)
        assert info["engine"] == (1 if info["panels"] > 0 else 0)
        assert int(got[0]) == want, (n, int(got[0]), want, info)


def motif_triplet(rng, lens, at):
    """Unrelated random sequences sharing one conserved stretch, placed in the
    longest sequence at fraction `at` of its length (0: its start, 1: its end),
    so that the best local alignment lies in the first half, the second half,
    or across the middle."""
    t = [synth.uniform_seq(rng, m) for m in lens]
    ax = int(np.argmax(lens))
    m = min(40, *[max(n, 1) for n in lens])
    motif = synth.uniform_seq(rng, m)
    for q, n in enumerate(lens):
        if n < m:
            continue
        pos = int(round(at * (n - m))) if q == ax else int(rng.integers(0, n - m + 1))
        t[q][pos:pos + m] = synth.fix_length(rng, synth.mutate(rng, motif, 0.05), m) if q != ax else motif
    return tuple(t)


def test_lone_local_triplet_half_split(torch_cuda):
    # A lone local triplet under automatic options is scored by halves: the
    # best of the two halves' own bests and of the paths crossing the middle
    # plane. Compared with the classic split engine and the oracle where the
    # best alignment sits in the first half, in the second, or across the
    # middle, on unrelated and related triplets, odd lengths, ties for the
    # longest, empty and length-1 sequences, other scorings and replays.
    rng = np.random.default_rng(47)
    sc = ts.scoring(kind=ts.LOCAL)
    cases = []
    for n in ((300, 120, 140), (257, 257, 90), (129, 40, 66)):
        for at in (0.0, 0.5, 1.0):
            cases.append(motif_triplet(rng, n, at))
    cases += [tuple(synth.uniform_seq(rng, m) for m in n)
              for n in ((256, 40, 33), (300, 0, 0), (0, 311, 7), (1, 1, 400), (64, 333, 1))]
    cases += [synth.mutated_triplet(rng, max(n), 0.1, lens=n) for n in ((290, 290, 290), (513, 200, 150))]
    for q, t in enumerate(cases):
        n = tuple(int(s.size) for s in t)
        want = oracle.score(t, kind=oracle.LOCAL)
        say(f"local half split #{q} lens={n}")
        got_half, info = run_plan(torch_cuda, [t], sc)
        got_classic, _ = run_plan(torch_cuda, [t], sc, engine=1)
        assert int(got_half[0]) == int(got_classic[0]) == want, (q, n, int(got_half[0]), int(got_classic[0]), want)
        assert ts.score(t, sc) == want
    for trial in range(3):
        sub = pins.random_symmetric_sub(rng, -4, 5)
        gap = int(rng.integers(-5, 1))
        t = motif_triplet(rng, (200, 150, 170), float(rng.uniform(0, 1)))
        say(f"local half split scoring trial {trial} gap={gap}")
        got, _ = run_plan(torch_cuda, [t], ts.scoring(sub=sub, gap=gap, kind=ts.LOCAL))
        assert int(got[0]) == oracle.score(t, sub, gap, kind=oracle.LOCAL)
    t = motif_triplet(rng, (400, 380, 390), 0.9)
    say("local half split graph replays")
    outs, _ = run_plan(torch_cuda, [t], sc, use_graph=True, reps=4)
    assert all(int(o[0]) == oracle.score(t, kind=oracle.LOCAL) for o in outs)


def test_which_lone_triplets_take_the_halves(torch_cuda):
    # The halves path sweeps two triplets (twice the panel jobs of the
    # classic split, here 2 x 4 against 4): global from 128 residues on, local
    # from 128 to 2047 (an explicit threshold lifts that cap), semi-global
    # never. Scores against the oracle either way.
    rng = np.random.default_rng(49)
    cases = [(ts.GLOBAL, oracle.GLOBAL, 2048, 0, 8), (ts.LOCAL, oracle.LOCAL, 2047, 0, 8),
             (ts.LOCAL, oracle.LOCAL, 2048, 0, 4), (ts.LOCAL, oracle.LOCAL, 2048, 128, 8),
             (ts.SEMI_GLOBAL, oracle.SEMI_GLOBAL, 2047, 0, 4)]
    for kind, okind, n0, hmin, panels in cases:
        t = synth.mutated_triplet(rng, n0, 0.1, lens=(n0, 40, 40))
        lens, off, words = ts.pack_batch([t])
        plan = ts.Plan(lens, off, sc=ts.scoring(kind=kind), half_split_min=hmin)
        d_words = torch_cuda.from_numpy(words.view(np.int32)).cuda()
        d_scores = torch_cuda.full((1,), -7, dtype=torch_cuda.int32, device="cuda")
        say(f"lone triplet kind={kind} n0={n0} half_split_min={hmin}")
        plan.run(d_words, d_scores)
        torch_cuda.cuda.synchronize()
        info = plan.info()
        plan.close()
        assert info["panels"] == panels, (kind, n0, hmin, info)
        assert int(d_scores.cpu()[0]) == oracle.score(t, kind=okind)


@pytest.mark.parametrize("name,kind,okind", KINDS, ids=KIND_IDS)
def test_mixed_batch_and_few_wavefronts(torch_cuda, name, kind, okind):
    # One large triplet is split (its panels fold their bests), the rest are
    # swept whole, in one launch; then the same with fewer wavefronts than
    # panel jobs.
    rng = np.random.default_rng(44)
    trips = related(rng, 1, 220, 220) + related(rng, 40, 5, 60)
    want = want_of(trips, okind)
    sc = ts.scoring(kind=kind)
    say(f"{name} mixed batch")
    got, info = run_plan(torch_cuda, trips, sc)
    assert info["engine"] == 2, info
    assert (got == want).all(), report(trips, got, want)
    for grid in (1, 3, 7):
        say(f"{name} split grid={grid}")
        got, info = run_plan(torch_cuda, trips[:1], sc, engine=1, grid=grid)
        assert info["grid"] == grid
        assert int(got[0]) == want[0]


@pytest.mark.parametrize("name,kind,okind", KINDS, ids=KIND_IDS)
def test_repeated_runs_and_graph_replays(torch_cuda, name, kind, okind):
    # The per-triplet folds are reset before every run, eager or replayed.
    rng = np.random.default_rng(45)
    trips = related(rng, 2, 150, 190) + related(rng, 10, 10, 50)
    want = want_of(trips, okind)
    sc = ts.scoring(kind=kind)
    for use_graph in (False, True):
        say(f"{name} repeated runs graph={use_graph}")
        outs, _ = run_plan(torch_cuda, trips, sc, engine=1, use_graph=use_graph, reps=4)
        for got in outs:
            assert (got == want).all(), report(trips, got, want)


@pytest.mark.parametrize("name,kind,okind", KINDS, ids=KIND_IDS)
def test_random_scoring_schemes(torch_cuda, name, kind, okind):
    rng = np.random.default_rng(46)
    for trial in range(5):
        sub = pins.random_symmetric_sub(rng, -4, 5)
        gap = int(rng.integers(-5, 1))
        sc = ts.scoring(sub=sub, gap=gap, kind=kind)
        trips = related(rng, 20, 0, 80) + [tuple(synth.uniform_seq(rng, int(m))
                                                 for m in rng.integers(0, 80, 3)) for _ in range(10)]
        want = want_of(trips, okind, sub, gap)
        say(f"{name} scoring trial {trial} gap={gap}")
        got, _ = run_plan(torch_cuda, trips, sc, engine=0)
        assert (got == want).all(), report(trips, got, want)
        got1, _ = run_plan(torch_cuda, trips[:1], sc, engine=1)
        assert int(got1[0]) == want[0]


def load_golden(workload, name):
    path = os.path.join(GOLDEN, f"{workload}_{name.replace('-', '')}.json")
    with open(path) as f:
        g = json.load(f)
    assert g["kind"] == name
    return g


@pytest.mark.parametrize("name,kind,okind", KINDS, ids=KIND_IDS)
def test_single_1k(torch_cuda, name, kind, okind):
    # Full size: 1024 x 1000 x 1048, split over the whole device (the
    # configuration the benchmark times), against the stored oracle score
    # and, through trioseq_score, end to end.
    g = load_golden("single_1k", name)
    wl = synth.single_1k()
    assert [[int(s.size) for s in t] for t in wl.triplets] == g["lengths"]
    t = wl.triplets[0]
    say(f"{name} single_1k")
    got, info = run_plan(torch_cuda, [t], ts.scoring(kind=kind))
    assert info["engine"] == 1
    assert int(got[0]) == g["scores"][0]
    assert ts.score(t, ts.scoring(kind=kind)) == g["scores"][0]


@pytest.mark.parametrize("name,kind,okind", KINDS, ids=KIND_IDS)
def test_single_4k(torch_cuda, name, kind, okind):
    # Full size: 4096 x 4000 x 4150 (6.8e10 cells) as the benchmark runs it.
    g = load_golden("single_4k", name)
    wl = synth.single_4k()
    assert [[int(s.size) for s in t] for t in wl.triplets] == g["lengths"]
    say(f"{name} single_4k")
    got, info = run_plan(torch_cuda, wl.triplets, ts.scoring(kind=kind))
    assert int(got[0]) == g["scores"][0]


@pytest.mark.parametrize("name,kind,okind", KINDS, ids=KIND_IDS)
def test_batch_8192(torch_cuda, name, kind, okind):
    # Full size: all 8192 triplets in one launch, every score against the
    # stored oracle scores, for the library's default shape and for each
    # shape the autotuner may pick for the kind (eager and graph replay).
    g = load_golden("batch_8192", name)
    wl = synth.batch_8192()
    assert [[int(s.size) for s in t] for t in wl.triplets] == g["lengths"]
    want = np.asarray(g["scores"])
    sc = ts.scoring(kind=kind)
    for tile, graph in (((0, 0), False), ((8, 4), True), ((4, 4), False)):
        say(f"{name} batch_8192 tile={tile} graph={graph}")
        got, _ = run_plan(torch_cuda, wl.triplets, sc, tile=tile, use_graph=graph)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, [(int(q), int(got[q]), int(want[q])) for q in bad[:5]]


@pytest.mark.parametrize("name,kind,okind", KINDS, ids=KIND_IDS)
def test_autotune_is_parity_gated_for_kinds(torch_cuda, name, kind, okind):
    # The autotuner tries every shape compiled for the kind (4x4 and 8x4 here),
    # keeps only candidates whose scores equal the reference configuration's,
    # and a plan created afterwards with default options takes its choice.
    torch = torch_cuda
    rng = np.random.default_rng(48)
    trips = related(rng, 80, 20, 160)
    lens, off, words = ts.pack_batch(trips)
    d_words = torch.from_numpy(words.view(np.int32)).cuda()
    sc = ts.scoring(kind=kind)
    say(f"{name} autotune")
    res = ts.autotune(lens, off, d_words, sc=sc, reps=1)
    assert res["tried"] >= 2 and res["rejected"] == 0
    got, info = run_plan(torch, trips, sc)
    assert (info["tile_rows"], info["tile_cols"]) == (res["best"]["tile_rows"], res["best"]["tile_cols"])
    assert (got == want_of(trips, okind)).all()
