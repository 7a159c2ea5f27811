"""Writes the oracle's scores for the fixed-seed workloads to tests/golden/.

Calls only ``oracle`` (the CPU triple loop) and the seeded input generator;
nothing here touches the GPU path. Each output file records the workload,
its seed and the scoring, so the GPU tests can compare bit for bit without
re-running multi-minute oracle computations.

    python tests/golden/make_golden.py single_128 single_1k batch_8192 single_4k
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2605_28400_amd import synth  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def main(names):
    for name in names:
        w = synth.WORKLOADS[name]()
        t0 = time.time()
        scores = oracle.score_batch(w.triplets, oracle.DEFAULT_SUB, oracle.DEFAULT_GAP,
                                    threads=os.cpu_count())
        dt = time.time() - t0
        rec = {
            "workload": w.name, "generator": name, "seed": w.seed,
            "scoring": {"match": 1, "mismatch": -1, "gap": -2},
            "lengths": [[int(s.size) for s in t] for t in w.triplets],
            "cells": w.total_cells, "scores": [int(v) for v in scores],
            "oracle_seconds": round(dt, 2), "oracle_threads": os.cpu_count(),
        }
        path = os.path.join(OUT, f"{name}.json")
        with open(path, "w") as f:
            json.dump(rec, f, separators=(",", ":"))
        print(f"{name}: {len(scores)} scores, {w.total_cells:.3e} cells, {dt:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(synth.WORKLOADS))
