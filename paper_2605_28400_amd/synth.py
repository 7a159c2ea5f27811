"""Seeded synthetic DNA triplet generators.

This module only draws random residues. It holds none of the alignment
arithmetic, so both the CPU oracle (tests) and the GPU path (library,
bench) can take their inputs from it without sharing any scoring code.

Residues are integer codes 0..3 standing for A, C, G, T.

The paper benchmarks on simulated triplets of lengths 8..1024 (Section V-A,
Section V-E); those simulated datasets are not available, so the workloads
here are mutated-ancestor triplets of the same shape:

* an ancestor of i.i.d. uniform residues;
* three descendants made independently from it by one left-to-right pass:
  every ancestor position may start a deletion run, else it is copied with a
  substitution (to a uniformly chosen *different* residue) at the given rate;
  every position may also be followed by an inserted run of uniform residues;
  run lengths are geometric on {1, 2, ...} with p = 0.5;
* for workloads with fixed lengths, each descendant is truncated, or extended
  with uniform residues, to its stated length.

The random stream is numpy's PCG64 seeded with the workload seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ALPHABET = b"ACGT"


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_seq(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.integers(0, 4, size=int(n), dtype=np.uint8)


def mutate(rng: np.random.Generator, anc: np.ndarray, sub_rate: float,
           ins_rate: float = 0.01, del_rate: float = 0.01,
           geom_p: float = 0.5) -> np.ndarray:
    """One descendant of ``anc`` (see the module docstring for the process)."""
    n = int(anc.size)
    u_del = rng.random(n)
    u_sub = rng.random(n)
    u_ins = rng.random(n)
    shift = rng.integers(1, 4, size=n, dtype=np.uint8)
    out = anc.copy()
    subst = u_sub < sub_rate
    out[subst] = (out[subst] + shift[subst]) % 4
    keep = np.ones(n, dtype=bool)
    covered = -1
    for p in np.flatnonzero(u_del < del_rate):
        if p <= covered:
            continue
        run = int(rng.geometric(geom_p))
        keep[p:p + run] = False
        covered = p + run - 1
    ins_sites = np.flatnonzero(u_ins < ins_rate)
    if ins_sites.size == 0:
        return out[keep]
    pieces = []
    start = 0
    for p in ins_sites:
        pieces.append(out[start:p + 1][keep[start:p + 1]])
        pieces.append(uniform_seq(rng, int(rng.geometric(geom_p))))
        start = p + 1
    pieces.append(out[start:][keep[start:]])
    return np.concatenate(pieces).astype(np.uint8)


def fix_length(rng: np.random.Generator, seq: np.ndarray, n: int) -> np.ndarray:
    if seq.size >= n:
        return seq[:n].copy()
    return np.concatenate([seq, uniform_seq(rng, n - seq.size)])


def to_ascii(codes: np.ndarray) -> bytes:
    return np.frombuffer(ALPHABET, dtype=np.uint8)[codes].tobytes()


def from_ascii(text: bytes) -> np.ndarray:
    lut = np.full(256, 255, dtype=np.uint8)
    for c, ch in enumerate(b"ACGT"):
        lut[ch] = c
        lut[ch + 32] = c
    return lut[np.frombuffer(text, dtype=np.uint8)]


Triplet = tuple  # (np.ndarray, np.ndarray, np.ndarray) of uint8 codes


def cells(t: Triplet) -> int:
    return int(t[0].size) * int(t[1].size) * int(t[2].size)


def mutated_triplet(rng, anc_len, sub_rate, lens=None):
    anc = uniform_seq(rng, anc_len)
    seqs = [mutate(rng, anc, sub_rate) for _ in range(3)]
    if lens is not None:
        seqs = [fix_length(rng, s, n) for s, n in zip(seqs, lens)]
    return tuple(seqs)


@dataclass
class Workload:
    name: str
    triplets: list
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def total_cells(self) -> int:
        return sum(cells(t) for t in self.triplets)


def single_128(seed: int = 1) -> Workload:
    """Three independent uniform sequences of length 128."""
    rng = rng_for(seed)
    t = tuple(uniform_seq(rng, 128) for _ in range(3))
    return Workload("single_128x128x128", [t], seed)


def single_1k(seed: int = 2) -> Workload:
    """Mutated-ancestor triplet fixed to lengths 1024/1000/1048."""
    rng = rng_for(seed)
    t = mutated_triplet(rng, 1024, 0.05, lens=(1024, 1000, 1048))
    return Workload("single_1024x1000x1048", [t], seed)


def batch_8192(seed: int = 3, count: int = 8192) -> Workload:
    """Ancestor lengths uniform in [100, 400], substitution rate in [0.02, 0.15]."""
    rng = rng_for(seed)
    trips = []
    for _ in range(count):
        n = int(rng.integers(100, 401))
        rate = float(rng.uniform(0.02, 0.15))
        trips.append(mutated_triplet(rng, n, rate))
    return Workload(f"batch_{count}_len100-400", trips, seed)


def single_4k(seed: int = 4) -> Workload:
    """Mutated-ancestor triplet fixed to lengths 4096/4000/4150."""
    rng = rng_for(seed)
    t = mutated_triplet(rng, 4096, 0.05, lens=(4096, 4000, 4150))
    return Workload("single_4096x4000x4150", [t], seed)


def served_stream(seed: int = 5, count: int = 100_000):
    """Requests with log-uniform ancestor lengths in [64, 2048].

    Returns (workload, unit_gaps): ``unit_gaps`` are exponential
    inter-arrival draws of mean 1; divide by a rate (requests/s) to get a
    Poisson arrival process at that rate.
    """
    rng = rng_for(seed)
    lo, hi = math.log(64), math.log(2048)
    trips = []
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(lo, hi))))
        rate = float(rng.uniform(0.02, 0.15))
        trips.append(mutated_triplet(rng, n, rate))
    gaps = rng.exponential(1.0, size=count)
    return Workload(f"served_{count}_len64-2048", trips, seed), gaps


def served_mix(seed: int = 8) -> Workload:
    """A served round's mix: 60 requests with log-uniform ancestor lengths in
    [64, 512] and four long ones (ancestors of 1536, 1792, 1900 and 2048
    residues, the top of the served stream's range), in a seeded order;
    substitution rates uniform in [0.02, 0.15]."""
    rng = rng_for(seed)
    lo, hi = math.log(64), math.log(512)
    anc = [int(round(math.exp(rng.uniform(lo, hi)))) for _ in range(60)] + [1536, 1792, 1900, 2048]
    order = rng.permutation(len(anc))
    trips = [mutated_triplet(rng, anc[q], float(rng.uniform(0.02, 0.15))) for q in order]
    return Workload("served_mix_64_len64-2048", trips, seed)


def fuzz(seed: int, count: int, max_len: int, skewed: bool = True) -> list:
    """Random triplets with uniform lengths in [0, max_len] plus degenerate shapes."""
    rng = rng_for(seed)
    out = []
    for _ in range(count):
        lens = rng.integers(0, max_len + 1, size=3)
        out.append(tuple(uniform_seq(rng, int(n)) for n in lens))
    if skewed:
        m = max(max_len, 1)
        shapes = [(1, 1, m), (m, m, 0), (1, m, m), (0, 0, m), (0, 0, 0),
                  (m, 1, 1), (0, m, 1), (2, m, 3)]
        for s in shapes:
            out.append(tuple(uniform_seq(rng, n) for n in s))
        for n in (1, 7, m):
            x = uniform_seq(rng, n)
            out.append((x.copy(), x.copy(), x.copy()))
            out.append((np.zeros(n, np.uint8), np.ones(n, np.uint8),
                        np.full(n, 2, np.uint8)))
    return out


WORKLOADS = {
    "single_128": single_128,
    "single_1k": single_1k,
    "batch_8192": batch_8192,
    "single_4k": single_4k,
    "served_mix": served_mix,
}
