"""GPU tests of the continuous-batching server through the C ABI.

Every served score must equal the oracle's (and the score of the same triplet
scored alone); requests that arrive while others run are admitted into new
rounds that overlap on the device; bad requests fail alone.
"""
import json
import os
import sys
import threading
import time

import numpy as np
import pytest

import oracle
import paper_2605_28400_amd as ts
from paper_2605_28400_amd import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
INT32_MIN = -(1 << 31)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def mixed_requests(seed, count, lo=8, hi=160):
    rng = synth.rng_for(seed)
    out = []
    for _ in range(count):
        n = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        out.append(synth.mutated_triplet(rng, n, float(rng.uniform(0.02, 0.15))))
    return out


def test_served_scores_equal_alone_and_oracle(gpu):
    reqs = mixed_requests(31, 300)
    # A few large requests that the server splits into panel jobs.
    rng = synth.rng_for(32)
    reqs += [synth.mutated_triplet(rng, n, 0.05) for n in (700, 650)]
    want = oracle.score_batch(reqs)
    srv = ts.Server(max_len=1024, max_device_bytes=8 << 30)
    ids = []
    say(f"submitting {len(reqs)} requests in waves")
    for k, t in enumerate(reqs):
        ids.append(srv.submit(t))
        if k % 50 == 49:
            time.sleep(0.002)  # arrivals while earlier rounds are on the GPU
    got = {}
    for rid in ids:
        r = srv.wait(rid, timeout_s=60)
        assert r["status"] == 0, r
        got[rid] = r["score"]
    st = srv.stats()
    srv.close()
    scores = np.array([got[i] for i in ids])
    bad = np.flatnonzero(scores != want)
    assert bad.size == 0, [(int(q), int(scores[q]), int(want[q])) for q in bad[:5]]
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["rounds"] >= 2
    assert st["p50_ns"] > 0 and st["p99_ns"] >= st["p50_ns"]
    # Alone (plain per-triplet path) equals in the mix.
    for q in (0, 7, 150, len(reqs) - 1):
        assert ts.score(reqs[q]) == scores[q]


def test_concurrent_submitters_and_poll(gpu):
    reqs = mixed_requests(33, 240, lo=4, hi=120)
    want = oracle.score_batch(reqs)
    srv = ts.Server(max_len=256, max_batch=64, max_device_bytes=4 << 30)
    ids = [None] * len(reqs)

    def submit_range(k0):
        for q in range(k0, len(reqs), 4):
            ids[q] = srv.submit(reqs[q])
            time.sleep(0.0002)

    th = [threading.Thread(target=submit_range, args=(k,)) for k in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    results = {}
    t0 = time.time()
    while len(results) < len(reqs) and time.time() - t0 < 60:
        for r in srv.poll():
            results[r["id"]] = r
        time.sleep(0.001)
    srv.close()
    assert len(results) == len(reqs)
    for q, rid in enumerate(ids):
        assert results[rid]["status"] == 0 and results[rid]["score"] == want[q]


def test_bad_request_fails_alone_and_queue_limits(gpu):
    srv = ts.Server(max_len=64, max_queue=4, max_device_bytes=1 << 30)
    good = srv.submit(("ACGT", "ACG", "AGT"))
    with pytest.raises(ts.TrioseqError) as e:
        srv.submit(("ACGT", "ACXG", "A"))
    assert e.value.status == -2
    with pytest.raises(ts.TrioseqError) as e:
        srv.submit(("A" * 65, "A", "A"))
    assert e.value.status == -3
    assert srv.wait(good, timeout_s=30)["score"] == oracle.score(
        [synth.from_ascii(b"ACGT"), synth.from_ascii(b"ACG"), synth.from_ascii(b"AGT")])
    with pytest.raises(ts.TrioseqError) as e:
        srv.wait(good, timeout_s=1)  # already consumed
    assert e.value.status == -1
    # Fill the queue faster than it drains: BUSY appears, nothing is lost.
    ids, busy = [], 0
    for _ in range(400):
        try:
            ids.append(srv.submit(("ACGTACGT" * 8, "ACGT" * 16, "GT" * 32)))
        except ts.TrioseqError as err:
            assert err.status == -7
            busy += 1
    for rid in ids:
        assert srv.wait(rid, timeout_s=30)["status"] == 0
    srv.close()
    assert busy + len(ids) == 400


def test_destroy_with_work_in_flight(gpu):
    reqs = mixed_requests(34, 200, lo=50, hi=300)
    srv = ts.Server(max_len=512, max_device_bytes=4 << 30)
    for t in reqs:
        srv.submit(t)
    srv.close()  # drains queued and in-flight rounds, then frees everything
    with pytest.raises(Exception):
        srv.submit(reqs[0])


@pytest.mark.parametrize("kind,okind", [(ts.SEMI_GLOBAL, oracle.SEMI_GLOBAL),
                                        (ts.LOCAL, oracle.LOCAL)], ids=["semi-global", "local"])
def test_served_kinds_equal_oracle(gpu, kind, okind):
    # Served rounds of the semi-global and local kinds: whole-triplet jobs and
    # split requests (their panel bests fold across wavefronts) in one stream.
    reqs = mixed_requests(33, 200)
    rng = synth.rng_for(34)
    reqs += [synth.mutated_triplet(rng, n, 0.05) for n in (600, 520)]
    want = oracle.score_batch(reqs, kind=okind)
    srv = ts.Server(max_len=1024, sc=ts.scoring(kind=kind), max_device_bytes=8 << 30)
    say(f"serving {len(reqs)} requests, kind {kind}")
    ids = []
    for k, t in enumerate(reqs):
        ids.append(srv.submit(t))
        if k % 50 == 49:
            time.sleep(0.002)
    got = []
    for rid in ids:
        r = srv.wait(rid, timeout_s=60)
        assert r["status"] == 0, r
        got.append(r["score"])
    srv.close()
    assert np.array_equal(np.array(got), np.asarray(want)), \
        [(q, got[q], int(want[q])) for q in range(len(reqs)) if got[q] != want[q]][:5]


def test_served_long_requests_equal_oracle(gpu):
    # The top of the served stream's length range: four requests of 1500-2050
    # residues (split into panel jobs) among 60 short ones, every score
    # against the stored oracle scores, and alone (trioseq_score) = in the mix.
    with open(os.path.join(GOLDEN, "served_mix.json")) as f:
        g = json.load(f)
    wl = synth.served_mix()
    assert [[int(s.size) for s in t] for t in wl.triplets] == g["lengths"]
    longest = max(int(s.size) for t in wl.triplets for s in t)
    srv = ts.Server(max_len=longest, max_device_bytes=40 << 30)
    say(f"serving {len(wl.triplets)} requests up to {longest} residues")
    ids = []
    for k, t in enumerate(wl.triplets):
        ids.append(srv.submit(t))
        if k % 16 == 15:
            time.sleep(0.001)
    got = []
    for rid in ids:
        r = srv.wait(rid, timeout_s=90)
        assert r["status"] == 0, r
        got.append(r["score"])
    st = srv.stats()
    srv.close()
    assert got == g["scores"], [(q, got[q], g["scores"][q]) for q in range(len(got))
                                if got[q] != g["scores"][q]][:5]
    assert st["completed"] == len(ids) and st["gcups"] > 0
    for q, t in enumerate(wl.triplets):
        if max(s.size for s in t) > 1400:
            say(f"alone: request {q}")
            assert ts.score(t) == got[q]


@pytest.mark.parametrize("kind,okind", [(ts.GLOBAL, oracle.GLOBAL), (ts.LOCAL, oracle.LOCAL),
                                        (ts.SEMI_GLOBAL, oracle.SEMI_GLOBAL)],
                         ids=["global", "local", "semi-global"])
def test_rounds_of_one_request(gpu, kind, okind):
    # Each request waited for (and its round given time to end) before the
    # next is submitted, so every round holds one request and runs alone:
    # lone requests split into panel jobs over the whole device, for each
    # kind. Odd lengths, the longest on each axis, an empty sequence, and
    # local alignments at either end of the longest sequence.
    rng = synth.rng_for(37)
    reqs = [synth.mutated_triplet(rng, max(n), 0.08, lens=n)
            for n in ((300, 280, 290), (129, 200, 77), (90, 60, 257), (500, 0, 310), (127, 100, 90))]
    for at in (0.0, 1.0):
        t = [synth.uniform_seq(rng, n) for n in (400, 150, 170)]
        motif = synth.uniform_seq(rng, 40)
        t[0][int(at * 360):int(at * 360) + 40] = motif
        t[1][50:90] = motif
        t[2][60:100] = motif
        reqs.append(tuple(t))
    want = [oracle.score(t, kind=okind) for t in reqs]
    srv = ts.Server(max_len=512, sc=ts.scoring(kind=kind), max_device_bytes=4 << 30)
    got = []
    for q, t in enumerate(reqs):
        say(f"round of one request #{q} kind={kind} lens={[s.size for s in t]}")
        r = srv.wait(srv.submit(t), timeout_s=60)
        assert r["status"] == 0, r
        got.append(r["score"])
        time.sleep(0.01)
    st = srv.stats()
    srv.close()
    assert got == want, [(q, got[q], want[q]) for q in range(len(reqs)) if got[q] != want[q]]
    assert st["rounds"] == len(reqs)


@pytest.mark.parametrize("inflight", [1, 8])
def test_rounds_in_flight_setting(gpu, inflight):
    reqs = mixed_requests(35, 160, lo=8, hi=200)
    want = oracle.score_batch(reqs)
    srv = ts.Server(max_len=256, max_batch=32, max_device_bytes=2 << 30, max_inflight=inflight)
    say(f"max_inflight={inflight}")
    ids = [srv.submit(t) for t in reqs]
    got = [srv.wait(rid, timeout_s=60)["score"] for rid in ids]
    st = srv.stats()
    srv.close()
    assert got == [int(v) for v in want]
    assert st["rounds"] >= len(reqs) // 32


def test_rounds_in_flight_limit_rejected(gpu):
    with pytest.raises(ts.TrioseqError) as e:
        ts.Server(max_len=64, max_inflight=17)
    assert e.value.status == -1


def test_wait_that_gives_up_never_reports_a_wrong_score(gpu):
    # The kernels' waits for other wavefronts are bounded; a wait that gives up
    # lets the run finish, and the score must then be INT32_MIN (a served
    # request fails) rather than a value computed from stale faces. The
    # condition is forced from the host with a wait bound of a few
    # nanoseconds, so every wave still exits normally.
    torch = gpu
    rng = synth.rng_for(36)
    t = synth.mutated_triplet(rng, 300, 0.1, lens=(300, 290, 310))
    want = oracle.score(t)
    lens, off, words = ts.pack_batch([t])
    d_words = torch.from_numpy(words.view(np.int32)).cuda()
    seen = []
    ts.set_wait_limit(1)
    try:
        for engine in (1, -1):
            plan = ts.Plan(lens, off, engine=engine)
            for rep in range(3):
                d_score = torch.full((1,), -7, dtype=torch.int32, device="cuda")
                say(f"forced give-up engine={engine} rep={rep}")
                plan.run(d_words, d_score)
                torch.cuda.synchronize()
                seen.append(int(d_score.cpu()[0]))
            plan.close()
        srv = ts.Server(max_len=512, max_device_bytes=2 << 30)
        served = srv.wait(srv.submit(t), timeout_s=60)
        srv.close()
    finally:
        ts.set_wait_limit(0)
    assert all(v in (INT32_MIN, want) for v in seen), seen
    assert INT32_MIN in seen, seen
    assert served["status"] != 0 or served["score"] == want, served
    # Back at the default bound, the same triplet scores correctly.
    assert ts.score(t) == want
