"""Throughput benchmark of exact 3-way alignment scoring on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--kind global|semi-global|local]

A step is one scoring pass of the whole hot path over the workload's batch,
with the packed residues already resident in HBM. The default workload is the
batch of 8192 mutated-ancestor triplets with ancestor lengths 100-400
(1.75e11 cells in one persistent launch), the largest workload that is
measured on one GPU as a single step. Prints one JSON line: GCUPS (10^9 cell
updates/s, cells = a*b*c per triplet), the INT32 VALU roofline of the
dominant kernel, parity of every score against the oracle's stored scores,
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12 int32 lane-ops/s.
PEAK_INT32_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic VALU work per cell: 4 adds + 3 three-input maxima (the shifted
# recurrence of Eq. 1 with hoisted substitution terms). Local scoring adds the
# floor v = 0 and the running maximum over the tensor (one maximum each);
# semi-global adds maxima over the last slices only (O(n^2) cells).
OPS_PER_CELL_OF = {"global": 7, "semi-global": 7, "local": 9}
OPS_PER_CELL = OPS_PER_CELL_OF["global"]
# Packed pairs (two triplets per lane, one 16-bit half each): 5 packed
# additions and 3 packed three-input maxima serve two cell updates, so the
# floor is 4 VALU instructions per cell against the same 39.32e12 lane-
# instruction peak; local scoring adds a packed floor maximum and a packed
# running maximum per two cells.
OPS_PER_CELL_PACKED_OF = {"global": 4, "semi-global": 4, "local": 5}
OPS_PER_CELL_PACKED = OPS_PER_CELL_PACKED_OF["global"]

WORKLOADS = ("single_1k", "single_128", "batch_8192", "single_4k", "served", "traceback")

# HBM bytes per launch of the sweep kernel, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs scaled by the same counters on a plain 1 GiB copy (summaries
# with the commands are under profiles/). Each figure holds only for the kernel
# source it was measured on; for any other source the field is null.
# Keyed by (workload, kind, lane tile, path): the autotuner may pick another
# tile, and a lone global or local triplet under automatic options is scored by
# halves.
TRAFFIC = {
    ("batch_8192_len100-400", "global", "4x4", "batch-packed+lds-direct"): (4.8549e10, "121dba023671257b"),
    ("batch_8192_len100-400", "local", "4x4", "batch-packed"): (4.8426e10, "121dba023671257b"),
    ("batch_8192_len100-400", "semi-global", "4x4", "batch-packed"): (4.8503e10, "121dba023671257b"),
    ("single_1024x1000x1048", "global", "4x4", "halves"): (1.5255e9, "121dba023671257b"),
    ("single_4096x4000x4150", "global", "4x4", "halves"): (7.7745e10, "121dba023671257b"),
    ("single_128x128x128", "global", "4x4", "halves"): (5.8941e6, "121dba023671257b"),
    ("single_1024x1000x1048", "local", "4x4", "halves"): (1.6171e9, "121dba023671257b"),
    ("batch_8192_len100-400", "global", "8x4", "batch"): (7.2410e10, "5b986628d09c52c4"),
    ("single_1024x1000x1048", "global", "4x4", "split"): (1.5689e9, "5b986628d09c52c4"),
    ("single_4096x4000x4150", "global", "4x4", "split"): (7.9174e10, "5b986628d09c52c4"),
    ("single_1024x1000x1048", "local", "4x4", "split"): (1.6522e9, "5b986628d09c52c4"),
    ("batch_8192_len100-400", "local", "4x4", "batch"): (9.7230e10, "5b986628d09c52c4"),
    ("single_1024x1000x1048", "semi-global", "4x4", "split"): (1.6210e9, "5b986628d09c52c4"),
    ("batch_8192_len100-400", "semi-global", "8x4", "batch"): (7.3193e10, "5b986628d09c52c4"),
}


def scoring_path(trips, kind: str, engine: int, tile: str, packed: bool = False) -> str:
    """Which kernels a plan runs: "halves" (a lone global triplet whose longest
    sequence has at least 128 residues, or a local one with 128 to 2047, automatic
    engine, 4x4 tiles: its two halves swept concurrently with the last-slice plane
    variant, then met), "split" (panel jobs), "batch" (several triplets) or
    "batch-packed" (several triplets, two per lane in 16-bit halves)."""
    if len(trips) != 1:
        return "batch-packed" if packed else "batch"
    longest = max(s.size for s in trips[0])
    if (engine == -1 and tile in ("0x0", "4x4") and longest >= 128
            and (kind == "global" or (kind == "local" and longest < 2048))):
        return "halves"
    return "split"


def measured_traffic(workload_name: str, kind: str, tile: str, path: str):
    import hashlib
    entry = TRAFFIC.get((workload_name, kind, tile, path))
    if entry is None:
        return None
    src = os.path.join(ROOT, "paper_2605_28400_amd", "csrc", "sweep.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return entry[0] if sha == entry[1] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch_8192", choices=WORKLOADS)
    ap.add_argument("--kind", default="global", choices=tuple(OPS_PER_CELL_OF),
                    help="alignment kind (paper, Section II)")
    ap.add_argument("--tile", default="0x0", help="lane tile RJxRK (0x0 = library default)")
    ap.add_argument("--engine", type=int, default=-1)
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--requests", type=int, default=100_000, help="served: stream length")
    ap.add_argument("--load", type=float, default=0.8,
                    help="served: offered load as a fraction of measured batched throughput")
    ap.add_argument("--autotune", type=int, default=1,
                    help="batches: pick the tile shape with the parity-gated autotuner first (untimed)")
    ap.add_argument("--per-triplet-sample", type=int, default=256,
                    help="batches: also time this many triplets through the plain per-triplet path")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def golden_scores(name: str, kind: str):
    """The oracle's stored scores for a fixed-seed workload (written by
    tests/golden/make_golden.py, which calls only the oracle), or None."""
    fname = name if kind == "global" else f"{name}_{kind.replace('-', '')}"
    path = os.path.join(ROOT, "tests", "golden", f"{fname}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    return np.asarray(g["scores"], dtype=np.int64)


def host_cpu() -> dict:
    """The host's CPU model and logical CPU count (reported beside the oracle)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def cpu_baseline(workload, budget_s: float = 20.0, kind: str = "global"):
    """The oracle, as is, on a bounded sample of the workload (host cores)."""
    import oracle
    okind = {"global": oracle.GLOBAL, "semi-global": oracle.SEMI_GLOBAL, "local": oracle.LOCAL}[kind]
    from paper_2605_28400_amd import synth
    trips = workload.triplets
    cores = 1 if len(trips) == 1 else (os.cpu_count() or 1)
    if len(trips) == 1:
        t = trips[0]
        cells = synth.cells(t)
        if cells > 3e9:
            # A prefix of the sweep sequence: same shape class, bounded time.
            n0 = max(1, int(2e9 / (t[1].size * t[2].size)))
            t = (t[0][:n0], t[1], t[2])
            sample = f"first {n0} residues of the sweep sequence x full other two (1 thread)"
        else:
            sample = "the whole triplet (1 thread)"
        cells = synth.cells(t)
        t0 = time.perf_counter()
        score = oracle.score(t, kind=okind)
        dt = time.perf_counter() - t0
        return {"value": cells / dt / 1e9, "unit": "GCUPS", "cores": cores, "kind": "oracle",
                "sample": sample, "seconds": round(dt, 3), **host_cpu()}, score
    # Batched: as many triplets (in workload order) as fit the time budget
    # at the oracle's measured rate, on all host cores.
    probe = trips[:cores]
    t0 = time.perf_counter()
    oracle.score_batch(probe, threads=cores, kind=okind)
    rate = sum(synth.cells(t) for t in probe) / max(time.perf_counter() - t0, 1e-6)
    take, acc = 0, 0.0
    for t in trips:
        acc += synth.cells(t)
        take += 1
        if acc > rate * budget_s:
            break
    sample = trips[:take]
    cells = sum(synth.cells(t) for t in sample)
    t0 = time.perf_counter()
    oracle.score_batch(sample, threads=cores, kind=okind)
    dt = time.perf_counter() - t0
    return {"value": cells / dt / 1e9, "unit": "GCUPS", "cores": cores, "kind": "oracle",
            "sample": f"first {take} of {len(trips)} triplets on {cores} threads",
            "seconds": round(dt, 3), **host_cpu()}, None


def per_triplet(ts, torch, trips, sample: int, stream, ref_scores=None, spread: bool = False,
                sc=None):
    """The plain per-triplet path on the same GPU: one plan per triplet
    (inputs resident in HBM), built and warmed untimed, then one timed,
    synchronised run each; plans are freed one by one, so large triplets
    never hold their panel faces at the same time. `sample` triplets are
    taken from the front (or evenly spread over the list)."""
    idx = (np.linspace(0, len(trips) - 1, min(sample, len(trips))).astype(int) if spread
           else np.arange(min(sample, len(trips))))
    from paper_2605_28400_amd import synth
    busy, cells, alone = 0.0, 0.0, []
    for q in idx:
        t = trips[int(q)]
        lens, off, words = ts.pack_batch([t])
        plan = ts.Plan(lens, off, sc=sc)
        w = torch.from_numpy(words.view(np.int32)).cuda()
        d_score = torch.zeros(1, dtype=torch.int32, device="cuda")
        plan.run(w, d_score, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.run(w, d_score, stream)
        torch.cuda.synchronize()
        busy += time.perf_counter() - t0
        cells += synth.cells(t)
        alone.append(int(d_score.cpu()[0]))
        plan.close()
    rec = {"value": round(cells / busy / 1e9, 3), "unit": "GCUPS", "ms": round(busy * 1e3, 3),
           "sample": f"{len(idx)} triplets ({'spread over' if spread else 'first of'} {len(trips)}), "
                     "one plan each, one synchronised launch each"}
    if ref_scores is not None:
        rec["scores_equal"] = bool((np.array(alone) == np.asarray(ref_scores)[idx]).all())
    return rec


def served(args):
    """Poisson stream through the continuous-batching server.

    The offered rate is load x the server's closed-loop capacity on these
    requests (the first ones submitted all at once), in requests per second.
    Reports sustained GCUPS (cells of all requests / first submit to last
    result), the submit-to-result latency percentiles, and the plain
    per-triplet path on a sample of the same requests (whose scores must
    equal the served ones).
    """
    import torch
    import paper_2605_28400_amd as ts
    from paper_2605_28400_amd import synth
    sc = ts.scoring(kind=args.kind)
    ops = OPS_PER_CELL_OF[args.kind]
    print(f"generating {args.requests} requests", file=sys.stderr, flush=True)
    workload, gaps = synth.served_stream(count=args.requests)
    trips = workload.triplets
    cells_each = np.array([synth.cells(t) for t in trips], dtype=np.float64)
    cells = float(cells_each.sum())
    max_len = max(max(a.size, b.size, c.size) for a, b, c in trips)
    budget = 64 << 30
    # Closed-loop capacity on the first requests.
    calib = min(len(trips), max(200, len(trips) // 50))
    srv = ts.Server(max_len=max_len, sc=sc, max_device_bytes=budget)
    t0 = time.perf_counter()
    cids = [srv.submit(t) for t in trips[:calib]]
    for rid in cids:
        srv.wait(rid, timeout_s=600)
    cap = cells_each[:calib].sum() / (time.perf_counter() - t0)
    srv.close()
    rate = args.load * cap / cells_each.mean()
    print(f"capacity {cap / 1e9:.1f} GCUPS -> offered {rate:.1f} requests/s", file=sys.stderr, flush=True)
    srv = ts.Server(max_len=max_len, sc=sc, max_device_bytes=budget)
    arrivals = np.cumsum(gaps / rate)
    ids = []
    start = time.perf_counter()
    for k, t in enumerate(trips):
        delay = arrivals[k] - (time.perf_counter() - start)
        if delay > 0:
            time.sleep(delay)
        ids.append(srv.submit(t))
        if k % 5000 == 0:
            print(f"submitted {k}/{len(trips)}", file=sys.stderr, flush=True)
    res = {}
    last = 0
    for rid in ids:
        r = srv.wait(rid, timeout_s=600)
        res[rid] = r
        last = max(last, r["t_done_ns"])
    st = srv.stats()
    first = min(r["t_submit_ns"] for r in res.values())
    srv.close()
    served_s = (last - first) * 1e-9
    ok = all(r["status"] == 0 for r in res.values())
    served_scores = np.array([res[rid]["score"] for rid in ids])
    stream = torch.cuda.current_stream()
    alone = per_triplet(ts, torch, trips, args.per_triplet_sample, stream, served_scores, spread=True,
                        sc=sc)
    rec = {
        "metric": "GCUPS", "value": round(cells / served_s / 1e9, 3), "unit": "GCUPS", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(served_s * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": workload.name, "requests": len(trips), "cells": int(cells),
                   "seed": workload.seed, "arrivals": "Poisson", "rate_req_per_s": round(rate, 1),
                   "offered_load": args.load, "closed_loop_capacity_gcups": round(cap / 1e9, 3),
                   "kind": args.kind, "parallelism": "single GPU"},
        "latency_ms": {"p50": round(st["p50_ns"] / 1e6, 3), "p99": round(st["p99_ns"] / 1e6, 3)},
        "rounds": st["rounds"], "all_ok": ok, "per_triplet_path": alone,
        "roofline": {"bound": "alu", "achieved": round(cells * ops / served_s / 1e12, 3),
                     "peak": round(PEAK_INT32_TOPS, 2), "unit": "TOP/s",
                     "frac": round(cells * ops / served_s / 1e12 / PEAK_INT32_TOPS, 4),
                     "traffic": None, "ops_per_cell": ops,
                     "kernel": "k_sweep rounds (continuous batching), wall clock"},
    }
    print(json.dumps(rec), flush=True)


def traceback(args):
    """Optimal alignments (trioseq_align): the 1024 x 1000 x 1048 triplet,
    timed over K synchronous calls, and a batch of 100,000 length-8 triplets
    (the size the paper's traceback was measured at) through
    trioseq_align_batch. Cells are a*b*c of the aligned triplets."""
    import torch
    import paper_2605_28400_amd as ts
    from paper_2605_28400_amd import synth
    t = synth.single_1k().triplets[0]
    cells = float(synth.cells(t))
    for _ in range(args.warmup):
        ts.align(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rows, score = ts.align(t)
    wall = (time.perf_counter() - t0) / args.steps
    rng = synth.rng_for(6)
    short = [synth.mutated_triplet(rng, 8, 0.2, lens=(8, 8, 8)) for _ in range(100_000)]
    ts.align_batch(short[:1000])
    t0 = time.perf_counter()
    res = ts.align_batch(short)
    bwall = time.perf_counter() - t0
    # The library call alone: triplets and output buffers marshalled beforehand.
    import ctypes
    keep: list = []
    arr = (ts.Triplet * len(short))()
    for q, tr in enumerate(short):
        arr[q] = ts._triplet(tr, keep)
    buf = ctypes.create_string_buffer(3 * 24 * len(short))
    ncols = np.zeros(len(short), dtype=np.uint32)
    scores = np.zeros(len(short), dtype=np.int32)
    lwall = []
    for _ in range(3):
        t0 = time.perf_counter()
        ts.check(ts.lib().trioseq_align_batch(arr, len(short), ctypes.byref(ts.scoring()), buf,
                                              ncols.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                              scores.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                              None))
        lwall.append(time.perf_counter() - t0)
    lwall = min(lwall)
    assert [int(v) for v in scores] == [sc for _, sc in res]
    achieved = cells * OPS_PER_CELL / wall / 1e12
    rec = {
        "metric": "GCUPS", "value": round(cells / wall / 1e9, 3), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "traceback_single_1024x1000x1048", "call": "trioseq_align (host rows)",
                   "columns": len(rows[0]), "score": score, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_INT32_TOPS, 2),
                     "unit": "TOP/s", "frac": round(achieved / PEAK_INT32_TOPS, 4), "traffic": None,
                     "ops_per_cell": OPS_PER_CELL,
                     "kernel": "whole call (plane sweeps of every level, splits, leaves, copies)"},
        "batch_len8": {"triplets": len(short), "seconds": round(bwall, 4),
                       "alignments_per_s": round(len(short) / bwall, 1),
                       "gcups": round(512 * len(short) / bwall / 1e9, 4),
                       "call": "paper_2605_28400_amd.align_batch (Python strings in and out)",
                       "library_call": {"seconds": round(lwall, 4),
                                        "alignments_per_s": round(len(short) / lwall, 1),
                                        "gcups": round(512 * len(short) / lwall / 1e9, 4),
                                        "call": "trioseq_align_batch, host triplets in, host rows "
                                                "out, best of 3"}},
    }
    print(json.dumps(rec), flush=True)


def copy_calibration(mib: int) -> None:
    """A plain device-to-device copy of known size: reads and writes mib MiB per launch,
    so a byte counter's reading for it gives the counter's scale factor."""
    import torch
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n, "launches": 5}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.workload in ("served", "traceback"):
        if args.gpus != 1:
            print("bench.py runs on one GPU only.", file=sys.stderr)
            sys.exit(2)
        (served if args.workload == "served" else traceback)(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: every workload here is measured on a single "
              "MI355X; independent triplets would shard across GPUs without collectives, "
              "and no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2605_28400_amd as ts
    from paper_2605_28400_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    workload = synth.WORKLOADS[args.workload]()
    trips = workload.triplets
    sc = ts.scoring(kind=args.kind)
    ops = OPS_PER_CELL_OF[args.kind]
    lens, off, words = ts.pack_batch(trips)
    rj, rk = (int(v) for v in args.tile.split("x"))
    d_words = torch.from_numpy(words.view(np.int32)).cuda()
    tuned = None
    if len(trips) > 1 and args.autotune and (rj, rk) == (0, 0) and args.engine == -1:
        # Untimed: every configuration is timed on this batch and the fastest
        # one whose scores equal the reference configuration's is kept.
        tuned = ts.autotune(lens, off, d_words, sc=sc, reps=2)
    plan = ts.Plan(lens, off, sc=sc, engine=args.engine, tile=(rj, rk), use_graph=bool(args.graph))
    info = plan.info()
    packed = bool(info["packed"])
    path = scoring_path(trips, args.kind, args.engine, args.tile, packed)
    if packed:
        ops = OPS_PER_CELL_PACKED_OF[args.kind]
        # The plan takes the autotuner's choice, staging included.
        if tuned is not None and tuned["best"]["staging"] == 2:
            path += "+lds-direct"
    d_scores = torch.zeros(len(trips), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.run(d_words, d_scores, stream)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        plan.run(d_words, d_scores, stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_events = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))

    cells = float(workload.total_cells)
    ms_per_step = wall * 1e3 / args.steps
    gcups = cells / (ms_per_step * 1e-3) / 1e9
    achieved = cells * ops / (ms_events * 1e-3) / 1e12
    scores = d_scores.cpu().numpy()

    rec = {
        "metric": "GCUPS", "value": round(gcups, 3), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int16x2" if packed else "int32",
        "data": "synthetic",
        "config": {"workload": workload.name, "triplets": len(trips), "cells": int(cells),
                   "seed": workload.seed, "scoring": "match +1, mismatch -1, gap -2",
                   "kind": args.kind, "packed_pairs": packed,
                   "engine": ["whole-triplet", "split", "mixed"][info["engine"]], "path": path,
                   "tile": f"{info['tile_rows']}x{info['tile_cols']}", "grid": info["grid"],
                   "hip_graph": bool(args.graph), "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(PEAK_INT32_TOPS, 2), "unit": "TOP/s",
                     "frac": round(achieved / PEAK_INT32_TOPS, 4),
                     "traffic": measured_traffic(workload.name, args.kind,
                                                 f"{info['tile_rows']}x{info['tile_cols']}", path),
                     "kernel_ms": round(ms_events, 4), "ops_per_cell": ops,
                     # Eq. 1 counted as 7 sums and a 7-way maximum (13 two-input
                     # operations), each an int32 instruction.
                     "frac_13_ops_per_cell": round(cells * (OPS_PER_CELL_OF[args.kind] + 6)
                                                   / (ms_events * 1e-3) / 1e12
                                                   / PEAK_INT32_TOPS, 4),
                     "kernel": ("k_panel plane variant (two halves swept concurrently, two-wave "
                                "panel workgroups) + gather + meet; time of the whole plan run"
                                if path == "halves" else
                                "k_sweep_pk (persistent job queue of whole-triplet pairs, two "
                                "triplets per lane in 16-bit halves)" if packed else
                                ["k_sweep (persistent job queue, whole-triplet jobs)",
                                 "k_panel (persistent job queue, two-wave panel workgroups)",
                                 "k_sweep (persistent job queue, whole-triplet and panel jobs)"][info["engine"]])},
    }
    # End to end through the host API: validate and pack the host ASCII, upload,
    # lay out (or reuse this thread's cached layout), sweep, download. The C
    # array of triplets is built beforehand (Python marshalling is not timed).
    import ctypes
    arr, keep = ts.triplet_array(trips)
    e2e_scores = np.zeros(len(trips), dtype=np.int32)

    def e2e_call():
        ts.check(ts.lib().trioseq_score_batch(arr, len(trips), ctypes.byref(sc),
                                              e2e_scores.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                              None))
    e2e_call()
    t0 = time.perf_counter()
    e2e_call()
    e2e_s = time.perf_counter() - t0
    rec["end_to_end"] = {"value": round(cells / e2e_s / 1e9, 3), "unit": "GCUPS",
                         "ms": round(e2e_s * 1e3, 3),
                         "call": "trioseq_score_batch: host ASCII triplets in, host scores out "
                                 "(second call: the layout of the first is reused)",
                         "scores_equal": bool((e2e_scores == scores).all())}
    gold = golden_scores(args.workload, args.kind)
    if gold is not None:
        rec["parity_vs_oracle"] = bool(gold.shape == scores.shape and (gold == scores).all())
        rec["parity_scores_checked"] = int(gold.size)
    if tuned is not None:
        b = tuned["best"]
        rec["config"]["autotuned"] = {"tile": f"{b['tile_rows']}x{b['tile_cols']}",
                                      "waves_per_simd": b["waves_per_simd"] or "auto",
                                      "packed": b["packed"] == 2,
                                      "lane_exchange": "registers" if b["lane_exchange"] == 2 else "lds",
                                      "split_factor": b["split_factor"] or 4,
                                      "staging": "lds-direct" if b["staging"] == 2 else "registers",
                                      "tried": tuned["tried"], "rejected": tuned["rejected"]}
    if len(trips) > 1 and args.per_triplet_sample > 0:
        rec["per_triplet_path"] = per_triplet(ts, torch, trips, args.per_triplet_sample, stream,
                                              scores, sc=sc)
    if not args.no_cpu_baseline:
        cb, oracle_score = cpu_baseline(workload, kind=args.kind)
        rec["cpu_baseline"] = cb
        if oracle_score is not None and len(trips) == 1 and cb["sample"].startswith("the whole"):
            rec["parity_vs_oracle_live"] = bool(int(scores[0]) == oracle_score)
    print(json.dumps(rec), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
