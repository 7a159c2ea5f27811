"""Python binding of libtrioseq (exact 3-way alignment scores on MI355X: global,
semi-global and local).

Argument marshalling only: every step of the scoring path runs in the HIP
library (``libtrioseq.so``, built by ``build.py``). If the library is not
built, importing the binding's functions raises; there is no CPU fallback.
PyTorch is used only to own device buffers and to name HIP streams.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrioseq.so")

OK = 0
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "BAD_RESIDUE", -3: "TOO_LARGE", -4: "OVERFLOW",
          -5: "NOMEM", -6: "DEVICE", -7: "BUSY", -8: "TIMEOUT", -9: "CLOSED"}


class TrioseqError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


# Alignment kinds (values of trioseq_kind).
GLOBAL, SEMI_GLOBAL, LOCAL = 0, 1, 2
KINDS = {"global": GLOBAL, "semi-global": SEMI_GLOBAL, "local": LOCAL}


class Scoring(ctypes.Structure):
    _fields_ = [("sub", (ctypes.c_int32 * 4) * 4), ("gap", ctypes.c_int32), ("kind", ctypes.c_int32)]


class Triplet(ctypes.Structure):
    _fields_ = [("seq", ctypes.c_char_p * 3), ("len", ctypes.c_uint32 * 3)]


class PlanOptions(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("tile_cols", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("panel_group", ctypes.c_int32), ("lane_exchange", ctypes.c_int32),
                ("split_factor", ctypes.c_int32), ("half_split_min", ctypes.c_int32),
                ("packed", ctypes.c_int32), ("staging", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("tile_cols", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("panels", ctypes.c_int32), ("packed", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_uint64), ("cells", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("best", PlanOptions), ("best_ms", ctypes.c_double),
                ("reference_ms", ctypes.c_double), ("tried", ctypes.c_int32),
                ("rejected", ctypes.c_int32)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_device_bytes", ctypes.c_uint64),
                ("max_len", ctypes.c_uint32), ("max_queue", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("score", ctypes.c_int32), ("status", ctypes.c_int32),
                ("t_submit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("cells", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("p50_ns", ctypes.c_double), ("p99_ns", ctypes.c_double),
                ("gcups", ctypes.c_double)]


# Every symbol the C header declares (checked by the CPU test-suite).
EXPORTS = [
    "trioseq_scoring_simple", "trioseq_pack", "trioseq_packed_layout", "trioseq_score",
    "trioseq_score_batch", "trioseq_score_batch_packed", "trioseq_plan_create", "trioseq_plan_run", "trioseq_plan_get_info",
    "trioseq_plan_destroy", "trioseq_autotune", "trioseq_align", "trioseq_align_batch", "trioseq_serve_create", "trioseq_serve_submit", "trioseq_serve_poll",
    "trioseq_serve_wait", "trioseq_serve_stats_get", "trioseq_serve_get_stats", "trioseq_serve_destroy",
    "trioseq_set_wait_limit", "trioseq_last_error", "trioseq_version",
    "trioseq_score_batch_packed_noalloc", "trioseq_noalloc_scratch_bytes",
]

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2605_28400_amd/build.py (hipcc, gfx950)")
    # torch ships its own HIP runtime under the same soname: loaded first, it
    # also serves this library, so the process holds one runtime (loading the
    # library first would bring in a second one, and the first of the two to
    # open the device would own it).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    st = ctypes.c_int
    L.trioseq_scoring_simple.argtypes = [P(Scoring), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.trioseq_scoring_simple.restype = None
    L.trioseq_pack.argtypes = [ctypes.c_char_p, ctypes.c_uint32, P(ctypes.c_uint32)]
    L.trioseq_pack.restype = st
    L.trioseq_packed_layout.argtypes = [P(ctypes.c_uint32), ctypes.c_size_t, P(ctypes.c_uint64),
                                        P(ctypes.c_uint64)]
    L.trioseq_packed_layout.restype = st
    L.trioseq_score.argtypes = [P(Triplet), P(Scoring), P(ctypes.c_int32)]
    L.trioseq_score.restype = st
    L.trioseq_score_batch.argtypes = [P(Triplet), ctypes.c_size_t, P(Scoring), P(ctypes.c_int32),
                                      ctypes.c_void_p]
    L.trioseq_score_batch.restype = st
    L.trioseq_plan_create.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint64), ctypes.c_size_t,
                                      P(Scoring), P(PlanOptions), P(ctypes.c_void_p)]
    L.trioseq_plan_create.restype = st
    L.trioseq_plan_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.trioseq_plan_run.restype = st
    L.trioseq_plan_get_info.argtypes = [ctypes.c_void_p, P(PlanInfo)]
    L.trioseq_plan_get_info.restype = st
    L.trioseq_plan_destroy.argtypes = [ctypes.c_void_p]
    L.trioseq_plan_destroy.restype = st
    L.trioseq_autotune.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint64), ctypes.c_size_t,
                                   P(Scoring), ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   P(TuneResult)]
    L.trioseq_autotune.restype = st
    L.trioseq_serve_create.argtypes = [P(ServeConfig), P(Scoring), P(ctypes.c_void_p)]
    L.trioseq_serve_create.restype = st
    L.trioseq_serve_submit.argtypes = [ctypes.c_void_p, P(Triplet), P(ctypes.c_uint64)]
    L.trioseq_serve_submit.restype = st
    L.trioseq_serve_poll.argtypes = [ctypes.c_void_p, P(Result), ctypes.c_size_t, P(ctypes.c_size_t)]
    L.trioseq_serve_poll.restype = st
    L.trioseq_serve_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, P(Result), ctypes.c_int64]
    L.trioseq_serve_wait.restype = st
    L.trioseq_serve_get_stats.argtypes = [ctypes.c_void_p, P(ServeStats)]
    L.trioseq_serve_get_stats.restype = st
    L.trioseq_serve_stats_get.argtypes = [ctypes.c_void_p, P(ServeStats)]
    L.trioseq_serve_stats_get.restype = st
    L.trioseq_set_wait_limit.argtypes = [ctypes.c_uint64]
    L.trioseq_set_wait_limit.restype = None
    L.trioseq_serve_destroy.argtypes = [ctypes.c_void_p]
    L.trioseq_serve_destroy.restype = st
    L.trioseq_score_batch_packed.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_size_t, P(Scoring), ctypes.c_void_p,
                                             ctypes.c_void_p]
    L.trioseq_score_batch_packed.restype = st
    L.trioseq_score_batch_packed_noalloc.argtypes = L.trioseq_score_batch_packed.argtypes
    L.trioseq_score_batch_packed_noalloc.restype = st
    L.trioseq_noalloc_scratch_bytes.argtypes = []
    L.trioseq_noalloc_scratch_bytes.restype = ctypes.c_uint64
    L.trioseq_align.argtypes = [P(Triplet), P(Scoring), ctypes.c_char_p, ctypes.c_char_p,
                                ctypes.c_char_p, ctypes.c_uint32, P(ctypes.c_uint32),
                                P(ctypes.c_int32), ctypes.c_void_p]
    L.trioseq_align.restype = st
    L.trioseq_align_batch.argtypes = [P(Triplet), ctypes.c_size_t, P(Scoring), ctypes.c_char_p,
                                      P(ctypes.c_uint32), P(ctypes.c_int32), ctypes.c_void_p]
    L.trioseq_align_batch.restype = st
    L.trioseq_last_error.argtypes = []
    L.trioseq_last_error.restype = ctypes.c_char_p
    L.trioseq_version.argtypes = []
    L.trioseq_version.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int) -> None:
    if status != OK:
        raise TrioseqError(status, lib().trioseq_last_error().decode(errors="replace"))


def scoring(match: int = 1, mismatch: int = -1, gap: int = -2, sub=None, kind=GLOBAL) -> Scoring:
    """Scoring scheme; ``sub`` (4x4) overrides match/mismatch. ``kind`` is
    GLOBAL, SEMI_GLOBAL or LOCAL (or its name)."""
    s = Scoring()
    if sub is None:
        lib().trioseq_scoring_simple(ctypes.byref(s), match, mismatch, gap)
    else:
        sub = np.asarray(sub, dtype=np.int64)
        for x in range(4):
            for y in range(4):
                s.sub[x][y] = int(sub[x][y])
        s.gap = int(gap)
    s.kind = KINDS[kind] if isinstance(kind, str) else int(kind)
    return s


DEFAULT = None


def _default_scoring() -> Scoring:
    global DEFAULT
    if DEFAULT is None:
        DEFAULT = scoring()
    return DEFAULT


def _as_bytes(seq) -> bytes:
    if isinstance(seq, (bytes, bytearray)):
        return bytes(seq)
    if isinstance(seq, str):
        return seq.encode()
    arr = np.asarray(seq, dtype=np.uint8)
    return np.frombuffer(b"ACGT", dtype=np.uint8)[arr].tobytes()


def _triplet(t, keep: list) -> Triplet:
    tr = Triplet()
    for s in range(3):
        b = _as_bytes(t[s])
        keep.append(b)
        tr.seq[s] = b
        tr.len[s] = len(b)
    return tr


def score(triplet, sc: Scoring | None = None) -> int:
    """Exact SOP score of one triplet (ASCII strings/bytes or code arrays):
    global, semi-global or local as ``sc.kind`` says (global by default)."""
    keep: list = []
    tr = _triplet(triplet, keep)
    out = ctypes.c_int32()
    check(lib().trioseq_score(ctypes.byref(tr), ctypes.byref(sc or _default_scoring()), ctypes.byref(out)))
    return int(out.value)


def score_batch_packed(d_words, d_word_off, d_len, d_scores, n: int, sc: Scoring | None = None,
                       stream=None) -> None:
    """Scores of n triplets already in device memory (torch tensors or raw
    pointers): d_word_off (3n uint64), d_len (3n uint32), d_scores (n int32).
    Enqueued on ``stream`` (torch's current stream by default)."""
    ptr = lambda b: b.data_ptr() if hasattr(b, "data_ptr") else int(b)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    check(lib().trioseq_score_batch_packed(ctypes.c_void_p(ptr(d_words)), ctypes.c_void_p(ptr(d_word_off)),
                                           ctypes.c_void_p(ptr(d_len)), n,
                                           ctypes.byref(sc or _default_scoring()),
                                           ctypes.c_void_p(ptr(d_scores)), _stream_ptr(stream)))


def score_batch_packed_noalloc(d_words, d_word_off, d_len, d_scores, n: int,
                               sc: Scoring | None = None, stream=None) -> None:
    """As score_batch_packed, through the entry point that allocates no
    device memory (every buffer is carved from the library's fixed scratch
    array; calls on one GPU must not overlap in time)."""
    ptr = lambda b: b.data_ptr() if hasattr(b, "data_ptr") else int(b)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    check(lib().trioseq_score_batch_packed_noalloc(
        ctypes.c_void_p(ptr(d_words)), ctypes.c_void_p(ptr(d_word_off)), ctypes.c_void_p(ptr(d_len)), n,
        ctypes.byref(sc or _default_scoring()), ctypes.c_void_p(ptr(d_scores)), _stream_ptr(stream)))


def align(triplet, sc: Scoring | None = None, stream=None):
    """Optimal global alignment of one triplet: ((row0, row1, row2), score).
    Rows are strings of upper-case residues and '-' (the traceback)."""
    keep: list = []
    tr = _triplet(triplet, keep)
    cap = max(1, int(tr.len[0]) + int(tr.len[1]) + int(tr.len[2]))
    rows = [ctypes.create_string_buffer(cap) for _ in range(3)]
    n = ctypes.c_uint32()
    sco = ctypes.c_int32()
    check(lib().trioseq_align(ctypes.byref(tr), ctypes.byref(sc or _default_scoring()), rows[0],
                              rows[1], rows[2], cap, ctypes.byref(n), ctypes.byref(sco),
                              _stream_ptr(stream)))
    return tuple(r.raw[:n.value].decode() for r in rows), int(sco.value)


def align_batch(triplets, sc: Scoring | None = None, stream=None) -> list:
    """Optimal global alignments of many triplets, computed together:
    a list of ((row0, row1, row2), score)."""
    keep: list = []
    n = len(triplets)
    arr = (Triplet * max(n, 1))()
    caps = []
    for q, t in enumerate(triplets):
        arr[q] = _triplet(t, keep)
        caps.append(int(arr[q].len[0]) + int(arr[q].len[1]) + int(arr[q].len[2]))
    buf = ctypes.create_string_buffer(max(1, 3 * sum(caps)))
    ncols = np.zeros(max(n, 1), dtype=np.uint32)
    scores = np.zeros(max(n, 1), dtype=np.int32)
    check(lib().trioseq_align_batch(arr, n, ctypes.byref(sc or _default_scoring()), buf,
                                    ncols.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                    scores.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    _stream_ptr(stream)))
    raw = buf.raw
    out, base = [], 0
    for q in range(n):
        c, k = caps[q], int(ncols[q])
        out.append((tuple(raw[base + a * c: base + a * c + k].decode() for a in range(3)),
                    int(scores[q])))
        base += 3 * c
    return out


_ASCII = np.frombuffer(b"ACGT", dtype=np.uint8)


def triplet_array(triplets):
    """The C array of trioseq_triplet for many triplets, built in bulk: every
    sequence's ASCII goes into one buffer and the pointer and length fields
    are written through a numpy view of the array. Returns (array, buffer);
    the buffer must outlive every call that reads the array."""
    n = len(triplets)
    arr = (Triplet * max(n, 1))()
    if n == 0:
        return arr, None
    seqs = [s for t in triplets for s in t]
    if all(isinstance(s, np.ndarray) for s in seqs):
        lens = np.fromiter((s.size for s in seqs), dtype=np.int64, count=3 * n)
        codes = np.concatenate(seqs).astype(np.uint8, copy=False) if lens.sum() else np.zeros(0, np.uint8)
        data = _ASCII[codes] if codes.size else codes
    else:
        parts = [_as_bytes(s) for s in seqs]
        lens = np.fromiter((len(b) for b in parts), dtype=np.int64, count=3 * n)
        data = np.frombuffer(b"".join(parts), dtype=np.uint8)
    buf = np.empty(max(int(lens.sum()), 1), dtype=np.uint8)
    buf[:data.size] = data
    starts = np.zeros(3 * n, dtype=np.int64)
    np.cumsum(lens[:-1], out=starts[1:])
    view = np.frombuffer(arr, dtype=np.dtype({"names": ["seq", "len"], "formats": [("<u8", 3), ("<u4", 3)],
                                               "offsets": [Triplet.seq.offset, Triplet.len.offset],
                                               "itemsize": ctypes.sizeof(Triplet)}), count=n)
    view["seq"] = (buf.ctypes.data + starts).reshape(n, 3)
    view["len"] = lens.reshape(n, 3)
    return arr, buf


def score_batch(triplets, sc: Scoring | None = None, stream=None) -> np.ndarray:
    """Scores of many triplets in one persistent launch (synchronous)."""
    n = len(triplets)
    arr, keep = triplet_array(triplets)
    out = np.zeros(max(n, 1), dtype=np.int32)
    check(lib().trioseq_score_batch(arr, n, ctypes.byref(sc or _default_scoring()),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    _stream_ptr(stream)))
    return out[:n]


def _stream_ptr(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def pack(seq) -> np.ndarray:
    """2-bit packed words of one sequence (16 residues per uint32)."""
    b = _as_bytes(seq)
    words = np.zeros(max((len(b) + 15) // 16, 1), dtype=np.uint32)
    check(lib().trioseq_pack(b, len(b), words.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return words[:(len(b) + 15) // 16]


def pack_batch(triplets):
    """(lens[3n] uint32, word_off[3n] uint64, words uint32) in the default layout."""
    n = len(triplets)
    lens = np.array([[len(_as_bytes(s)) if not isinstance(s, np.ndarray) else s.size for s in t]
                     for t in triplets], dtype=np.uint32).reshape(3 * n)
    off = np.zeros(max(3 * n, 1), dtype=np.uint64)
    total = ctypes.c_uint64()
    check(lib().trioseq_packed_layout(lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), n,
                                      off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                      ctypes.byref(total)))
    words = np.zeros(max(int(total.value), 1), dtype=np.uint32)
    for q, t in enumerate(triplets):
        for s in range(3):
            w = pack(t[s])
            o = int(off[3 * q + s])
            words[o:o + w.size] = w
    return lens, off[:3 * n], words


class Plan:
    """Device-resident batch plan: ``run`` enqueues one scoring pass on a stream."""

    def __init__(self, lens, word_off=None, sc: Scoring | None = None, engine: int = -1,
                 tile=(0, 0), grid: int = 0, use_graph: bool = False, waves_per_simd: int = 0,
                 panel_group: int = 0, lane_exchange: int = 0, split_factor: int = 0,
                 half_split_min: int = 0, packed: int = 0, staging: int = 0):
        self.lens = np.ascontiguousarray(lens, dtype=np.uint32)
        self.n = self.lens.size // 3
        off_p = None
        if word_off is not None:
            self._off = np.ascontiguousarray(word_off, dtype=np.uint64)
            off_p = self._off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        opts = PlanOptions(engine, tile[0], tile[1], grid, 1 if use_graph else 0, waves_per_simd,
                           panel_group, lane_exchange, split_factor, half_split_min, packed, staging)
        self._h = ctypes.c_void_p()
        check(lib().trioseq_plan_create(self.lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                        off_p, self.n, ctypes.byref(sc or _default_scoring()),
                                        ctypes.byref(opts), ctypes.byref(self._h)))

    def run(self, d_words, d_scores, stream=None) -> None:
        """d_words / d_scores: device tensors (torch) or raw device pointers."""
        wp = d_words.data_ptr() if hasattr(d_words, "data_ptr") else int(d_words)
        sp = d_scores.data_ptr() if hasattr(d_scores, "data_ptr") else int(d_scores)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        check(lib().trioseq_plan_run(self._h, ctypes.c_void_p(wp), ctypes.c_void_p(sp),
                                     _stream_ptr(stream)))

    def info(self) -> dict:
        i = PlanInfo()
        check(lib().trioseq_plan_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in PlanInfo._fields_}

    def close(self) -> None:
        if self._h:
            lib().trioseq_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(lens, word_off, d_words, sc: Scoring | None = None, reps: int = 3,
             stream=None) -> dict:
    """Times every kernel configuration on this batch and remembers the fastest
    one whose scores equal the reference configuration's (see trioseq_autotune)."""
    lens = np.ascontiguousarray(lens, dtype=np.uint32)
    off = np.ascontiguousarray(word_off, dtype=np.uint64)
    wp = d_words.data_ptr() if hasattr(d_words, "data_ptr") else int(d_words)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    r = TuneResult()
    check(lib().trioseq_autotune(lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                 off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                 lens.size // 3, ctypes.byref(sc or _default_scoring()),
                                 ctypes.c_void_p(wp), reps, _stream_ptr(stream), ctypes.byref(r)))
    best = {f: getattr(r.best, f) for f, _ in PlanOptions._fields_}
    return {"best": best, "best_ms": r.best_ms, "reference_ms": r.reference_ms,
            "tried": r.tried, "rejected": r.rejected}


def version() -> str:
    return lib().trioseq_version().decode()


def set_wait_limit(ns: int = 0) -> None:
    """Bound on the kernels' waits for other wavefronts, for launches and graph
    captures made afterwards (0 = the default of 2 s); see trioseq_set_wait_limit."""
    lib().trioseq_set_wait_limit(int(ns))


class Server:
    """Continuous-batching scoring server (one GPU, background device thread)."""

    def __init__(self, max_len: int = 2048, sc: Scoring | None = None, device: int = 0,
                 max_queue: int = 0, max_batch: int = 0, max_device_bytes: int = 0,
                 max_inflight: int = 0):
        cfg = ServeConfig(device, max_device_bytes, max_len, max_queue, max_batch, max_inflight)
        self._h = ctypes.c_void_p()
        check(lib().trioseq_serve_create(ctypes.byref(cfg), ctypes.byref(sc or _default_scoring()),
                                         ctypes.byref(self._h)))

    def submit(self, triplet) -> int:
        keep: list = []
        tr = _triplet(triplet, keep)
        rid = ctypes.c_uint64()
        check(lib().trioseq_serve_submit(self._h, ctypes.byref(tr), ctypes.byref(rid)))
        return int(rid.value)

    @staticmethod
    def _res(r: Result) -> dict:
        return {"id": int(r.id), "score": int(r.score), "status": int(r.status),
                "t_submit_ns": int(r.t_submit_ns), "t_done_ns": int(r.t_done_ns)}

    def poll(self, cap: int = 4096) -> list:
        buf = (Result * cap)()
        n = ctypes.c_size_t()
        check(lib().trioseq_serve_poll(self._h, buf, cap, ctypes.byref(n)))
        return [self._res(buf[k]) for k in range(n.value)]

    def wait(self, rid: int, timeout_s: float | None = None) -> dict:
        r = Result()
        t = -1 if timeout_s is None else int(timeout_s * 1e9)
        check(lib().trioseq_serve_wait(self._h, rid, ctypes.byref(r), t))
        return self._res(r)

    def stats(self) -> dict:
        st = ServeStats()
        check(lib().trioseq_serve_stats_get(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServeStats._fields_}

    def close(self) -> None:
        if self._h:
            check(lib().trioseq_serve_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
