"""CPU oracle for exact 3-way alignment scoring, global, semi-global and local
(test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this package. The library never imports it, and it imports nothing from the
library: the two share no code.

The arithmetic lives in ``trioseq_oracle.c`` (plain C triple loop over
Eq. 1 of the paper, Section II, in int64). This module compiles it with gcc
into ``liboracle.so`` next to the source and calls it through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trioseq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle (plain -O2, no hand vectorisation)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-pthread",
                        "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64p = ctypes.POINTER(ctypes.c_int64)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_score.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, u8p,
                                     ctypes.c_int64, i32p, ctypes.c_int32, i64p]
        lib.oracle_score.restype = ctypes.c_int
        lib.oracle_score_local.argtypes = lib.oracle_score.argtypes
        lib.oracle_score_local.restype = ctypes.c_int
        lib.oracle_score_semiglobal.argtypes = lib.oracle_score.argtypes
        lib.oracle_score_semiglobal.restype = ctypes.c_int
        lib.oracle_score_batch.argtypes = [u8p, i64p, i64p, ctypes.c_int64, i32p,
                                           ctypes.c_int32, i64p, ctypes.c_int, ctypes.c_int]
        lib.oracle_score_batch.restype = ctypes.c_int
        _lib = lib
    return _lib


def simple_sub(match: int, mismatch: int) -> np.ndarray:
    """4x4 substitution matrix with ``match`` on the diagonal, ``mismatch`` elsewhere."""
    m = np.full((4, 4), mismatch, dtype=np.int32)
    np.fill_diagonal(m, match)
    return m


# Scoring of every workload in this project: match +1, mismatch -1, and -2 for
# a residue against a gap (gap against gap scores 0 by definition).
DEFAULT_SUB = simple_sub(1, -1)
DEFAULT_GAP = -2


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


# Alignment kinds (the paper's Section II variants implemented here).
GLOBAL, SEMI_GLOBAL, LOCAL = 0, 1, 2


def score(triplet, sub=DEFAULT_SUB, gap: int = DEFAULT_GAP, kind: int = GLOBAL) -> int:
    """Optimal sum-of-pairs score of one triplet of codes 0..3: M[a][b][c]
    (global), the best cell on the last slices (semi-global) or the largest
    value of the local tensor (local)."""
    lib = _load()
    fn = {GLOBAL: lib.oracle_score, SEMI_GLOBAL: lib.oracle_score_semiglobal,
          LOCAL: lib.oracle_score_local}[kind]
    keep = [_u8(s) for s in triplet]
    sub = np.ascontiguousarray(sub, dtype=np.int32).reshape(16)
    out = ctypes.c_int64()
    rc = fn(keep[0][1], keep[0][0].size, keep[1][1], keep[1][0].size,
                          keep[2][1], keep[2][0].size,
                          sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(gap),
                          ctypes.byref(out))
    if rc != 0:
        raise MemoryError("oracle could not allocate its two slices")
    return int(out.value)


def score_batch(triplets, sub=DEFAULT_SUB, gap: int = DEFAULT_GAP, threads: int | None = None,
                kind: int = GLOBAL):
    """Scores of many triplets, one triplet per thread at a time."""
    lib = _load()
    n = len(triplets)
    lens = np.array([[s.size for s in t] for t in triplets], dtype=np.int64).reshape(3 * n)
    off = np.zeros(3 * n, dtype=np.int64)
    if n:
        off[1:] = np.cumsum(lens)[:-1]
    seqs = np.concatenate([np.asarray(s, dtype=np.uint8) for t in triplets for s in t]) \
        if n else np.zeros(1, np.uint8)
    seqs = np.ascontiguousarray(seqs if seqs.size else np.zeros(1, np.uint8))
    sub = np.ascontiguousarray(sub, dtype=np.int32).reshape(16)
    out = np.zeros(max(n, 1), dtype=np.int64)
    if threads is None:
        threads = os.cpu_count() or 1
    i64p = ctypes.POINTER(ctypes.c_int64)
    rc = lib.oracle_score_batch(seqs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                off.ctypes.data_as(i64p), lens.ctypes.data_as(i64p), n,
                                sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(gap),
                                out.ctypes.data_as(i64p), int(threads), int(kind))
    if rc != 0:
        raise MemoryError("oracle could not allocate its slices")
    return out[:n]
