"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and rejects bad input before any device call (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2605_28400_amd as ts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trioseq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(trioseq_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = ts.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert sorted(ts.EXPORTS) == names


def test_version_string():
    assert "gfx950" in ts.version()


def test_pack_layout_and_bits():
    w = ts.pack("ACGTACGTACGTACGTT")
    assert w.dtype == np.uint32 and w.size == 2
    # A=0 C=1 G=2 T=3, residue p at bits 2*(p%16).
    want0 = sum(c << (2 * p) for p, c in enumerate([0, 1, 2, 3] * 4))
    assert int(w[0]) == want0 and int(w[1]) == 3
    assert ts.pack("acgt").tolist() == ts.pack("ACGT").tolist()
    assert ts.pack("").size == 0


def test_packed_layout_offsets():
    lens, off, words = ts.pack_batch([("A" * 17, "", "C" * 16), ("G", "T" * 33, "A")])
    assert lens.tolist() == [17, 0, 16, 1, 33, 1]
    assert off.tolist() == [0, 2, 2, 3, 4, 7]
    assert words.size == 8


def _status(fn):
    with pytest.raises(ts.TrioseqError) as e:
        fn()
    return e.value.status


def test_bad_residue_rejected():
    assert _status(lambda: ts.pack("ACGN")) == -2
    assert _status(lambda: ts.score(("ACGT", "ACXT", "A"))) == -2
    assert "triplet 1" in str(pytest.raises(ts.TrioseqError, ts.score_batch,
                                            [("A", "C", "G"), ("A", "-", "G")]).value)


def test_pack_error_leaves_words_untouched():
    L = ts.lib()
    words = (ctypes.c_uint32 * 3)(7, 8, 9)
    seq = b"ACGT" * 8 + b"ACGN"
    assert L.trioseq_pack(seq, len(seq), words) == -2
    assert list(words) == [7, 8, 9]
    assert b"position 35" in L.trioseq_last_error()
    ok = b"TGCA" * 9
    assert L.trioseq_pack(ok, len(ok), words) == 0
    assert list(words) == [int(w) for w in ts.pack(ok.decode())]


def test_large_batch_validation_names_the_first_bad_triplet():
    # Large enough to be packed by several host threads: the message still
    # names the first bad triplet and sequence in batch order, and nothing
    # is written to the scores.
    rng = np.random.default_rng(3)
    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
    trips = [[acgt[rng.integers(0, 4, 150)].tobytes() for _ in range(3)] for _ in range(3000)]
    trips[2999][0] = b"N" + trips[2999][0][1:]
    trips[1700][2] = trips[1700][2][:-1] + b"x"
    trips[2200][1] = b"-" + trips[2200][1][1:]
    arr, keep = ts.triplet_array([tuple(t) for t in trips])
    out = np.full(len(trips), 5, dtype=np.int32)
    L = ts.lib()
    r = L.trioseq_score_batch(arr, len(trips), ctypes.byref(ts.scoring()),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None)
    assert r == -2
    assert L.trioseq_last_error() == b"triplet 1700, sequence 2: pack: character at position 149 is not ACGT"
    assert (out == 5).all()


def test_asymmetric_matrix_rejected():
    sub = np.full((4, 4), -1)
    np.fill_diagonal(sub, 1)
    sub[0, 1] = 2
    assert _status(lambda: ts.score(("A", "C", "G"), ts.scoring(sub=sub, gap=-2))) == -1


def test_byte_range_of_terms_rejected():
    assert _status(lambda: ts.score(("A", "C", "G"), ts.scoring(1, -1, gap=-70))) == -1
    assert _status(lambda: ts.score(("A", "C", "G"), ts.scoring(130, -1, gap=0))) == -1


def test_overflow_bound_rejected():
    # (a+b+c) * max(sub - 2*gap) must stay below 2^27.
    long, short = "A" * 1_200_000, "A" * 10
    assert _status(lambda: ts.score((long, long, short), ts.scoring(100, -1, gap=-10))) == -4


def test_too_large_rejected():
    L = ts.lib()
    lens = np.array([20000, 20000, 20000], dtype=np.uint32)
    h = ctypes.c_void_p()
    st = L.trioseq_plan_create(lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), None, 1,
                               ctypes.byref(ts.scoring()), None, ctypes.byref(h))
    assert st == -3


def test_null_pointers_rejected():
    L = ts.lib()
    assert L.trioseq_score(None, None, None) == -1
    out = ctypes.c_int32(123)
    tr = ts.Triplet()
    tr.len[0] = 3
    tr.seq[0] = None
    assert L.trioseq_score(ctypes.byref(tr), ctypes.byref(ts.scoring()), ctypes.byref(out)) == -1
    assert out.value == 123  # untouched on error
    assert L.trioseq_plan_create(None, None, 1, ctypes.byref(ts.scoring()), None, None) == -1
    assert L.trioseq_plan_run(None, None, None, None) == -1
    assert L.trioseq_autotune(None, None, 1, ctypes.byref(ts.scoring()), None, 1, None, None) == -1
    assert b"NULL" in L.trioseq_last_error() or L.trioseq_last_error()


def test_bad_plan_options_rejected():
    L = ts.lib()
    lens = np.array([3, 3, 3], dtype=np.uint32)
    h = ctypes.c_void_p()
    for opts in [ts.PlanOptions(5, 0, 0, 0, 0, 0), ts.PlanOptions(-1, 3, 3, 0, 0, 0),
                 ts.PlanOptions(-1, 0, 0, -4, 0, 0), ts.PlanOptions(-1, 4, 4, 0, 0, 3)]:
        assert L.trioseq_plan_create(lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), None, 1,
                                     ctypes.byref(ts.scoring()), ctypes.byref(opts),
                                     ctypes.byref(h)) == -1


def test_bad_kinds_rejected():
    # Validation happens before any device work.
    L = ts.lib()
    assert _status(lambda: ts.score(("A", "C", "G"), ts.scoring(kind=3))) == -1
    assert _status(lambda: ts.score(("A", "C", "G"), ts.scoring(kind=-1))) == -1
    # Semi-global and local scoring need gap <= 0.
    for kind in (ts.SEMI_GLOBAL, ts.LOCAL):
        assert _status(lambda: ts.score(("A", "C", "G"), ts.scoring(2, -1, gap=1, kind=kind))) == -1
    # ... and 4 x 4 or 8 x 4 tiles at two waves per SIMD.
    lens = np.array([3, 3, 3], dtype=np.uint32)
    h = ctypes.c_void_p()
    for kind in (ts.SEMI_GLOBAL, ts.LOCAL):
        for opts in [ts.PlanOptions(-1, 4, 8, 0, 0, 2), ts.PlanOptions(-1, 4, 4, 0, 0, 4),
                     ts.PlanOptions(-1, 8, 4, 0, 0, 4)]:
            assert L.trioseq_plan_create(lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), None,
                                         1, ctypes.byref(ts.scoring(kind=kind)), ctypes.byref(opts),
                                         ctypes.byref(h)) == -1
    assert ts.KINDS == {"global": 0, "semi-global": 1, "local": 2}
    assert ts.scoring(kind="local").kind == ts.LOCAL


def test_align_rejects_bad_input_before_device_work():
    L = ts.lib()
    keep = []
    tr = ts._triplet(("ACG", "AC", "G"), keep)
    rows = [ctypes.create_string_buffer(8) for _ in range(3)]
    n, sco = ctypes.c_uint32(77), ctypes.c_int32(123)
    args = lambda sc, cap: (ctypes.byref(tr), ctypes.byref(sc), rows[0], rows[1], rows[2], cap,
                            ctypes.byref(n), ctypes.byref(sco), None)
    assert L.trioseq_align(*args(ts.scoring(kind=ts.LOCAL), 8)) == -1      # global only
    assert L.trioseq_align(*args(ts.scoring(), 5)) == -1                   # cap < 3 + 2 + 1
    assert L.trioseq_align(None, ctypes.byref(ts.scoring()), rows[0], rows[1], rows[2], 8,
                           ctypes.byref(n), ctypes.byref(sco), None) == -1
    bad = ts._triplet(("ACX", "A", "A"), keep)
    assert L.trioseq_align(ctypes.byref(bad), ctypes.byref(ts.scoring()), rows[0], rows[1], rows[2],
                           8, ctypes.byref(n), ctypes.byref(sco), None) == -2
    assert n.value == 77 and sco.value == 123  # untouched on error


def test_align_batch_rejects_bad_input():
    L = ts.lib()
    n, s = ctypes.c_uint32(), ctypes.c_int32()
    assert L.trioseq_align_batch(None, 1, ctypes.byref(ts.scoring()), None, ctypes.byref(n),
                                 ctypes.byref(s), None) == -1
    keep = []
    arr = (ts.Triplet * 1)(ts._triplet(("AC", "A", "G"), keep))
    buf = ctypes.create_string_buffer(12)
    assert L.trioseq_align_batch(arr, 1, ctypes.byref(ts.scoring(kind=ts.SEMI_GLOBAL)), buf,
                                 ctypes.byref(n), ctypes.byref(s), None) == -1
    assert ts.align_batch([]) == []


def test_score_batch_packed_rejects_bad_input():
    L = ts.lib()
    assert L.trioseq_score_batch_packed(None, None, None, 3, ctypes.byref(ts.scoring()), None, None) == -1
    assert L.trioseq_score_batch_packed(None, None, None, 3, None, None, None) == -1
    assert L.trioseq_score_batch_packed(None, None, None, 0, ctypes.byref(ts.scoring()), None, None) == 0


def test_missing_library_fails_loudly(tmp_path):
    # No CPU fallback: without the built library every scoring call raises.
    import subprocess
    import sys as _sys
    code = (
        "import paper_2605_28400_amd as ts\n"
        f"ts.LIB_PATH = {str(tmp_path / 'absent.so')!r}\n"
        "ts._lib = None\n"
        "try:\n"
        "    ts.score(('ACGT', 'ACG', 'AC'))\n"
        "except ImportError as e:\n"
        "    print('raised', e)\n"
        "else:\n"
        "    print('no error')\n")
    out = subprocess.run([_sys.executable, "-c", code], capture_output=True, text=True,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert "raised" in out.stdout and "absent.so" in out.stdout, out.stdout + out.stderr


# The calls of the boundary as first proposed for this library (the paper's
# problem statement: sequences, substitution scores, gap; Section II, and the
# host pipeline of Section IV, Approach Overview).
BOUNDARY = ["trioseq_scoring_simple", "trioseq_score", "trioseq_score_batch",
            "trioseq_score_batch_packed", "trioseq_serve_create", "trioseq_serve_submit",
            "trioseq_serve_poll", "trioseq_serve_wait", "trioseq_serve_stats_get",
            "trioseq_serve_destroy", "trioseq_last_error"]


def test_boundary_calls_declared_and_exported():
    L = ts.lib()
    names = declared_functions()
    for name in BOUNDARY:
        assert name in names and hasattr(L, name), name


STRUCTS = {
    "trioseq_scoring": ts.Scoring, "trioseq_triplet": ts.Triplet,
    "trioseq_plan_options": ts.PlanOptions, "trioseq_plan_info": ts.PlanInfo,
    "trioseq_tune_result": ts.TuneResult, "trioseq_serve_config": ts.ServeConfig,
    "trioseq_result": ts.Result, "trioseq_serve_stats": ts.ServeStats,
}


def test_binding_structs_match_the_header(tmp_path):
    # A C program built against include/trioseq.h prints every field's offset
    # and each struct's size; the ctypes mirrors must agree.
    import subprocess
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "trioseq.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    want = {}
    for line in out:
        if line:
            cname, field, value = line.split()
            want[(cname, field)] = int(value)
    for cname, cls in STRUCTS.items():
        assert ctypes.sizeof(cls) == want[(cname, "size")], cname
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == want[(cname, field)], (cname, field)
