"""GPU parity at the size limits of the ABI.

The swept sequence of a triplet may be up to 16384 residues (its per-slice
lookup shifts live in LDS); the other two may be longer when the host can put
a sequence of at most 16384 on the sweep axis. These cases take every kind,
the split and whole engines, a batch that mixes a limit-size triplet with
small ones, and the traceback, against the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2605_28400_amd as ts
from paper_2605_28400_amd import synth

pytestmark = pytest.mark.gpu
MAX = 16384


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run(torch, trips, sc, engine):
    lens, off, words = ts.pack_batch(trips)
    plan = ts.Plan(lens, off, sc=sc, engine=engine)
    d_words = torch.from_numpy(words.view(np.int32)).cuda()
    d_scores = torch.full((len(trips),), -7, dtype=torch.int32, device="cuda")
    plan.run(d_words, d_scores)
    torch.cuda.synchronize()
    info = plan.info()
    plan.close()
    return d_scores.cpu().numpy(), info


@pytest.mark.parametrize("kind,okind", [(ts.GLOBAL, oracle.GLOBAL), (ts.SEMI_GLOBAL, oracle.SEMI_GLOBAL),
                                        (ts.LOCAL, oracle.LOCAL)], ids=["global", "semi-global", "local"])
def test_longest_sweep_sequence(gpu, kind, okind):
    rng = np.random.default_rng(71)
    big = synth.mutated_triplet(rng, 60, 0.1, lens=(MAX, 48, 40))
    small = [synth.mutated_triplet(rng, int(n), 0.1) for n in rng.integers(5, 60, 12)]
    sc = ts.scoring(kind=kind)
    want = np.asarray(oracle.score_batch([big] + small, kind=okind))
    for engine in (0, 1):
        say(f"kind {kind} ({MAX}, 48, 40) engine {engine}")
        got, _ = run(gpu, [big], sc, engine)
        assert int(got[0]) == want[0]
    say(f"kind {kind} mixed batch with ({MAX}, 48, 40)")
    got, info = run(gpu, [big] + small, sc, -1)
    assert (got == want).all()


def test_two_sequences_past_the_sweep_limit(gpu):
    # Only the third sequence fits the sweep axis; the host must choose it.
    rng = np.random.default_rng(72)
    t = (synth.uniform_seq(rng, MAX + 3000), synth.uniform_seq(rng, MAX + 100),
         synth.uniform_seq(rng, 3))
    want = oracle.score(t)
    for engine in (-1, 0, 1):
        say(f"lengths (19384, 16484, 3) engine {engine}")
        got, info = run(gpu, [t], ts.scoring(), engine)
        assert int(got[0]) == want


def test_all_sequences_past_the_limit_rejected(gpu):
    t = ("A" * (MAX + 1),) * 3
    with pytest.raises(ts.TrioseqError) as e:
        ts.score(t)
    assert e.value.status == -3
    with pytest.raises(ts.TrioseqError) as e:
        ts.align(("A" * (MAX + 1), "A", "A"))
    assert e.value.status == -3


def test_traceback_of_the_longest_sequence(gpu):
    rng = np.random.default_rng(73)
    t = synth.mutated_triplet(rng, 40, 0.1, lens=(MAX, 24, 20))
    say(f"align ({MAX}, 24, 20)")
    rows, score = ts.align(t)
    assert score == oracle.score(t)
    letters = {c: q for q, c in enumerate("ACGT")}
    for q in range(3):
        assert [letters[ch] for ch in rows[q] if ch != "-"] == [int(v) for v in t[q]]
