"""The allocation-free entry point against trioseq_score_batch_packed.

trioseq_score_batch_packed_noalloc carves every device buffer from the
library's fixed scratch array. Its scores must equal those of
trioseq_score_batch_packed on the same device inputs (integers: equality),
on two calls in a row, the second with a smaller input, for a batch of whole
triplets, a batch holding split triplets, a lone global or local triplet
(scored by halves) and the semi-global and local kinds; inputs beyond the scratch limits are
rejected before anything is launched.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2605_28400_amd as ts
from paper_2605_28400_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def device_batch(torch, trips):
    lens, off, words = ts.pack_batch(trips)
    return (torch.from_numpy(words.view(np.int32)).cuda(),
            torch.from_numpy(off.astype(np.uint64).view(np.int64)).cuda(),
            torch.from_numpy(lens.astype(np.uint32).view(np.int32)).cuda())


def both(torch, trips, sc=None):
    """(scores of the allocating call, scores of the allocation-free call)."""
    d_words, d_off, d_len = device_batch(torch, trips)
    n = len(trips)
    ref = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    got = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    ts.score_batch_packed(d_words, d_off, d_len, ref, n, sc)
    torch.cuda.synchronize()
    ts.score_batch_packed_noalloc(d_words, d_off, d_len, got, n, sc)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def mixed(seed, count, lo, hi):
    rng = synth.rng_for(seed)
    out = []
    for _ in range(count):
        anc = int(rng.integers(lo, hi + 1))
        out.append(synth.mutated_triplet(rng, anc, float(rng.uniform(0.02, 0.15))))
    return out


def test_scratch_size_is_stated():
    assert ts.lib().trioseq_noalloc_scratch_bytes() == 256 << 20


@pytest.mark.parametrize("kind", [ts.GLOBAL, ts.SEMI_GLOBAL, ts.LOCAL])
def test_batches_twice_second_smaller(torch_cuda, kind):
    sc = ts.scoring(kind=kind)
    # First call: 300 triplets of 20..260 residues plus one of ~6e7 cells,
    # which the automatic layout splits into panel jobs; second call: a
    # smaller batch of shorter triplets (the scratch keeps the first call's
    # contents).
    first = mixed(51, 300, 20, 260) + mixed(52, 1, 380, 400)
    second = mixed(53, 40, 5, 90)
    for name, trips in (("first", first), ("second", second)):
        say(f"noalloc kind={kind} {name} n={len(trips)}")
        ref, got = both(torch_cuda, trips, sc)
        bad = np.flatnonzero(ref != got)
        assert bad.size == 0, [(int(q), int(ref[q]), int(got[q])) for q in bad[:5]]
    okind = {ts.GLOBAL: oracle.GLOBAL, ts.SEMI_GLOBAL: oracle.SEMI_GLOBAL, ts.LOCAL: oracle.LOCAL}[kind]
    want = [oracle.score(t, kind=okind) for t in second[:8]]
    assert got[:8].tolist() == want


@pytest.mark.parametrize("kind", [ts.GLOBAL, ts.LOCAL])
def test_lone_triplets_twice_second_smaller(torch_cuda, kind):
    # A lone global or local triplet is scored by halves (gather, two plane
    # sweeps, the meeting reduction; local scoring also folds the halves' own
    # bests); then a smaller lone triplet, then the empty and one-residue
    # shapes.
    sc = ts.scoring(kind=kind)
    okind = {ts.GLOBAL: oracle.GLOBAL, ts.LOCAL: oracle.LOCAL}[kind]
    rng = synth.rng_for(54)
    big = synth.mutated_triplet(rng, 300, 0.05, lens=(300, 288, 310))
    small = synth.mutated_triplet(rng, 70, 0.05, lens=(70, 64, 77))
    for trips in ([big], [small], [(small[0], small[1][:0], small[2])], [(small[0][:1],) * 3]):
        say(f"noalloc lone kind={kind} lens={[s.size for s in trips[0]]}")
        ref, got = both(torch_cuda, trips, sc)
        assert got.tolist() == ref.tolist()
        if trips[0][0].size == 300:
            assert got.tolist() == [oracle.score(trips[0], kind=okind)]
    assert got.tolist() == [oracle.score(trips[0], kind=okind)]


def test_beyond_the_scratch_is_rejected(torch_cuda):
    torch = torch_cuda
    # The lone 1024 x 1000 x 1048 triplet's panel faces need about 0.6 GB.
    trips = synth.single_1k().triplets
    d_words, d_off, d_len = device_batch(torch, trips)
    out = torch.full((1,), -5, dtype=torch.int32, device="cuda")
    say("noalloc oversize")
    with pytest.raises(ts.TrioseqError) as ei:
        ts.score_batch_packed_noalloc(d_words, d_off, d_len, out, 1)
    assert ei.value.status == -3 and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert out.cpu().tolist() == [-5]
    # The entry point still works after a rejection.
    small = mixed(55, 5, 30, 60)
    ref, got = both(torch, small)
    assert got.tolist() == ref.tolist()
