"""Planted mistakes in the oracle must fail the pins.

Each case edits one line of the oracle's C source (a dropped term, a wrong
sign, a wrong index, a transposed operand, a wrong base value), builds the
edited copy in a temporary directory, and checks that the brute-force and
closed-form pins reject it. This shows the pins are strong enough to catch
the mistakes they are meant to catch. Only CPU code is built and run.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "trioseq_oracle.c")

MUTANTS = {
    "drop_triple_bc_term": (
        "pair(sub, x, y) + pair(sub, x, z) + pair(sub, y, z);",
        "pair(sub, x, y) + pair(sub, x, z);"),
    "gap_sign": (
        "v = prev[j * row + k] + g + g;", "v = prev[j * row + k] + g - g;"),
    "wrong_index_ij_move": (
        "v = prev[(j - 1) * row + k] + pair(sub, s0[i - 1], s1[j - 1]) + g + g;",
        "v = prev[j * row + k] + pair(sub, s0[i - 1], s1[j - 1]) + g + g;"),
    "transposed_operand_ik_move": (
        "pair(sub, s0[i - 1], s2[k - 1]) + g + g;",
        "pair(sub, s1[j > 0 ? j - 1 : 0], s2[k - 1]) + g + g;"),
    "prev_instead_of_cur_jk_move": (
        "v = cur[(j - 1) * row + (k - 1)] + pair(sub, s1[j - 1], s2[k - 1]) + g + g;",
        "v = prev[(j - 1) * row + (k - 1)] + pair(sub, s1[j - 1], s2[k - 1]) + g + g;"),
    "base_value": ("cur[0] = 0;", "cur[0] = 1;"),
    "drop_k_single_move": (
        "v = cur[j * row + (k - 1)] + g + g;", "v = cur[j * row + (k - 1)] + g + g - 1000;"),
    "single_gap_not_doubled": (
        "v = cur[(j - 1) * row + k] + g + g;", "v = cur[(j - 1) * row + k] + g;"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-pthread", "-o", str(so),
                    str(path)], check=True)
    lib = ctypes.CDLL(str(so))
    u8p, i32p, i64p = (ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32),
                       ctypes.POINTER(ctypes.c_int64))
    lib.oracle_score.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, u8p, ctypes.c_int64,
                                 i32p, ctypes.c_int32, i64p]

    def score(trip, sub, gap):
        arrs = [np.ascontiguousarray(s, np.uint8) for s in trip]
        sub = np.ascontiguousarray(sub, np.int32).reshape(16)
        out = ctypes.c_int64()
        lib.oracle_score(*[x for a in arrs for x in (a.ctypes.data_as(u8p), a.size)],
                         sub.ctypes.data_as(i32p), gap, ctypes.byref(out))
        return out.value

    return score


def _pins_pass(score) -> bool:
    rng = np.random.default_rng(1234)
    for trial in range(40):
        trip = [rng.integers(0, 4, size=int(n)).astype(np.uint8) for n in rng.integers(0, 4, 3)]
        sub = oracle.DEFAULT_SUB if trial % 2 else pins.random_symmetric_sub(rng)
        best, _ = pins.enumerate_alignments(trip, sub, -2)
        if score(trip, sub, -2) != best:
            return False
    x = rng.integers(0, 4, size=9).astype(np.uint8)
    if score([x, x, x], oracle.DEFAULT_SUB, -2) != 27:
        return False
    return True


def test_unmodified_source_passes(tmp_path):
    assert _pins_pass(_build(tmp_path, "identity", "cur[0] = 0;", "cur[0] = 0;"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    assert not _pins_pass(_build(tmp_path, name, old, new))


# Planted mistakes in the local variant, caught by its own pins (brute force
# over substring triples, identical sequences).
LOCAL_MUTANTS = {
    "local_no_zero_floor": ("int64_t m = 0; /* v = 0: the eighth candidate */",
                            "int64_t m = i + j + k ? -4000000 : 0;"),
    "local_score_not_tracked": ("top = m > top ? m : top;", "top = top;"),
    "local_single_gap_once": ("const int64_t twogap = 2 * (int64_t)gap;",
                              "const int64_t twogap = (int64_t)gap;"),
    "local_jk_move_from_last_slice": (
        "cand = here[(j - 1) * w + k - 1] + pair(sub, y, z) + twogap;",
        "cand = last[(j - 1) * w + k - 1] + pair(sub, y, z) + twogap;"),
    "local_drop_triple_move": (
        "cand = last[(j - 1) * w + k - 1] + (pair(sub, x, y) + pair(sub, x, z)) + pair(sub, y, z);",
        "cand = -4000000;"),
}


def _build_local(tmp_path, name, old, new, fn="oracle_score_local"):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-pthread", "-o", str(so),
                    str(path)], check=True)
    lib = ctypes.CDLL(str(so))
    u8p, i32p, i64p = (ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32),
                       ctypes.POINTER(ctypes.c_int64))
    f = getattr(lib, fn)
    f.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, u8p, ctypes.c_int64, i32p,
                  ctypes.c_int32, i64p]

    def score(trip, sub, gap):
        arrs = [np.ascontiguousarray(s, np.uint8) for s in trip]
        sub = np.ascontiguousarray(sub, np.int32).reshape(16)
        out = ctypes.c_int64()
        f(*[x for a in arrs for x in (a.ctypes.data_as(u8p), a.size)],
          sub.ctypes.data_as(i32p), gap, ctypes.byref(out))
        return out.value

    return score


def _local_pins_pass(score) -> bool:
    from tests.test_oracle_local import local_brute
    rng = np.random.default_rng(4321)
    memo = {}
    for trial in range(30):
        trip = [rng.integers(0, 4, size=int(n)).astype(np.uint8) for n in rng.integers(0, 3, 3)]
        sub = oracle.DEFAULT_SUB if trial % 2 else pins.random_symmetric_sub(rng)
        if score(trip, sub, -2) != local_brute(trip, sub, -2, memo):
            return False
    x = rng.integers(0, 4, size=9).astype(np.uint8)
    return score([x, x, x], oracle.DEFAULT_SUB, -2) == 27


def test_unmodified_local_source_passes(tmp_path):
    assert _local_pins_pass(_build_local(tmp_path, "local_identity", "top = m > top ? m : top;",
                                         "top = m > top ? m : top;"))


@pytest.mark.parametrize("name", sorted(LOCAL_MUTANTS))
def test_local_mutant_is_caught(tmp_path, name):
    old, new = LOCAL_MUTANTS[name]
    assert not _local_pins_pass(_build_local(tmp_path, name, old, new))


# Plausible mistakes in the semi-global variant (each must fail its pins).
SEMI_MUTANTS = {
    "semi_axes_from_moves": ("if ((i == 0) + (j == 0) + (k == 0) >= 2) {",
                             "if (i + j + k == 0) {"),
    "semi_last_slice_i_only": ("if ((i == a || j == b || k == c) && m > answer) answer = m;",
                               "if (i == a && m > answer) answer = m;"),
    "semi_whole_tensor": ("if ((i == a || j == b || k == c) && m > answer) answer = m;",
                          "if (m > answer) answer = m;"),
    "semi_faces_zero_too": ("if ((i == 0) + (j == 0) + (k == 0) >= 2) {",
                            "if ((i == 0) + (j == 0) + (k == 0) >= 1) {"),
    "semi_ik_move_wrong_residue": ("t = older[j * stride + (k - 1)] + gg + pair(sub, x, z);",
                                   "t = older[j * stride + (k - 1)] + gg + pair(sub, y, z);"),
    "semi_triple_from_this_slice": (
        "t = older[(j - 1) * stride + (k - 1)] + pair(sub, y, z) + pair(sub, x, y) + pair(sub, x, z);",
        "t = newer[(j - 1) * stride + (k - 1)] + pair(sub, y, z) + pair(sub, x, y) + pair(sub, x, z);"),
}


def _semi_pins_pass(score) -> bool:
    from tests.test_oracle_semiglobal import semi_brute
    rng = np.random.default_rng(8765)
    memo = {}
    for trial in range(40):
        trip = [rng.integers(0, 4, size=int(n)).astype(np.uint8) for n in rng.integers(0, 4, 3)]
        sub = oracle.DEFAULT_SUB if trial % 2 else pins.random_symmetric_sub(rng)
        gap = (-2, -1, 0)[trial % 3]
        if score(trip, sub, gap) != semi_brute(trip, sub, gap, memo):
            return False
    # The two hand-derived cases of tests/test_oracle_semiglobal.py.
    ac, c = np.array([0, 1], np.uint8), np.array([1], np.uint8)
    if score([ac, ac, c], oracle.DEFAULT_SUB, -2) != 0:
        return False
    ag, at = np.array([0, 2], np.uint8), np.array([0, 3], np.uint8)
    if score([ag, at, ac], oracle.DEFAULT_SUB, -2) != 0:
        return False
    x = rng.integers(0, 4, size=9).astype(np.uint8)
    return score([x, x, x], oracle.DEFAULT_SUB, -2) == 27


def test_unmodified_semiglobal_source_passes(tmp_path):
    line = "if ((i == a || j == b || k == c) && m > answer) answer = m;"
    assert _semi_pins_pass(_build_local(tmp_path, "semi_identity", line, line,
                                        fn="oracle_score_semiglobal"))


@pytest.mark.parametrize("name", sorted(SEMI_MUTANTS))
def test_semiglobal_mutant_is_caught(tmp_path, name):
    old, new = SEMI_MUTANTS[name]
    assert not _semi_pins_pass(_build_local(tmp_path, name, old, new, fn="oracle_score_semiglobal"))
