"""Host-side pieces of bench.py, checked without a GPU: the one-GPU contract,
the scoring-path classification that keys the measured HBM traffic, and the
rule that a traffic figure holds only for the kernel source it was measured
on."""
import hashlib
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def seqs(*lens):
    return tuple(np.zeros(n, dtype=np.uint8) for n in lens)


def test_more_than_one_gpu_exits_with_a_message():
    for extra in ([], ["--workload", "served"], ["--workload", "traceback"]):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", *extra],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2
        assert "one GPU" in r.stderr
        assert r.stdout == ""


def test_scoring_path():
    one_big, one_small = [seqs(128, 100, 90)], [seqs(127, 100, 90)]
    assert bench.scoring_path(one_big, "global", -1, "0x0") == "halves"
    assert bench.scoring_path(one_big, "global", -1, "4x4") == "halves"
    assert bench.scoring_path(one_big, "local", -1, "0x0") == "halves"
    assert bench.scoring_path([seqs(2047, 10, 10)], "local", -1, "0x0") == "halves"
    assert bench.scoring_path([seqs(2048, 10, 10)], "local", -1, "0x0") == "split"
    assert bench.scoring_path([seqs(2048, 10, 10)], "global", -1, "0x0") == "halves"
    # Below the half-split threshold, semi-global, a forced engine or tile.
    assert bench.scoring_path(one_small, "global", -1, "0x0") == "split"
    assert bench.scoring_path(one_big, "semi-global", -1, "0x0") == "split"
    assert bench.scoring_path(one_big, "global", 1, "0x0") == "split"
    assert bench.scoring_path(one_big, "global", -1, "8x4") == "split"
    two = one_big + one_small
    assert bench.scoring_path(two, "global", -1, "0x0") == "batch"
    assert bench.scoring_path(two, "global", -1, "0x0", packed=True) == "batch-packed"


def test_traffic_holds_only_for_its_source():
    with open(os.path.join(ROOT, "paper_2605_28400_amd", "csrc", "sweep.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    for key, (value, src) in bench.TRAFFIC.items():
        got = bench.measured_traffic(*key)
        assert got == (value if src == sha else None), key
        assert value > 0
    assert bench.measured_traffic("no such workload", "global", "4x4", "batch") is None


def test_ops_per_cell_floors():
    # int32: 4 additions and 3 three-input maxima per cell (local adds the
    # floor and the running maximum); packed: 8 instructions per two cells.
    assert bench.OPS_PER_CELL_OF == {"global": 7, "semi-global": 7, "local": 9}
    assert bench.OPS_PER_CELL_PACKED_OF == {"global": 4, "semi-global": 4, "local": 5}
    assert abs(bench.PEAK_INT32_TOPS - 39.3216) < 1e-3
