"""Independent references used to pin the oracle (no DP over the 3-D tensor).

* ``enumerate_alignments`` builds every 3-row global alignment explicitly
  (each row is its sequence in order with gaps inserted, all rows of one
  length, no all-gap column) and scores it column by column with the
  sum-of-pairs definition of Section II. The maximum over all of them is the
  exact global score by definition.
* ``delannoy3`` counts those alignments with the plain 3-D Delannoy
  recurrence, a known closed count (D(n,n,n) = 1, 13, 409, 16081, 699121).
* ``nw`` is the textbook two-sequence Needleman-Wunsch score with linear
  gaps, used for the reductions that hold when one sequence is empty and for
  the Carrillo-Lipman pairwise upper bound (cited by the paper, Section III).
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np

GAP = -1  # marker for a gap in an explicit alignment row


def pair_score(x: int, y: int, sub, gap: int) -> int:
    if x == GAP and y == GAP:
        return 0
    if x == GAP or y == GAP:
        return gap
    return int(sub[x][y])


def column_sop(col, sub, gap) -> int:
    x, y, z = col
    return pair_score(x, y, sub, gap) + pair_score(x, z, sub, gap) + pair_score(y, z, sub, gap)


def _rows(seqs):
    """Yield explicit alignments as lists of columns (tuples of codes or GAP)."""
    a, b, c = (list(map(int, s)) for s in seqs)
    out = []

    def rec(i, j, k, cols):
        if i == len(a) and j == len(b) and k == len(c):
            yield list(cols)
            return
        for di, dj, dk in itertools.product((0, 1), repeat=3):
            if di + dj + dk == 0:
                continue
            if i + di > len(a) or j + dj > len(b) or k + dk > len(c):
                continue
            cols.append((a[i] if di else GAP, b[j] if dj else GAP, c[k] if dk else GAP))
            yield from rec(i + di, j + dj, k + dk, cols)
            cols.pop()

    yield from rec(0, 0, 0, out)


def enumerate_alignments(seqs, sub, gap):
    """(best score, number of alignments) over every explicit alignment."""
    best = None
    count = 0
    for cols in _rows(seqs):
        count += 1
        # Score from the materialised rows, column by column.
        rows = list(zip(*cols)) if cols else [(), (), ()]
        s = sum(column_sop((rows[0][p], rows[1][p], rows[2][p]), sub, gap)
                for p in range(len(cols)))
        if best is None or s > best:
            best = s
    return best, count


@lru_cache(maxsize=None)
def delannoy3(a: int, b: int, c: int) -> int:
    if a < 0 or b < 0 or c < 0:
        return 0
    if a == 0 and b == 0 and c == 0:
        return 1
    tot = 0
    for di, dj, dk in itertools.product((0, 1), repeat=3):
        if di + dj + dk:
            tot += delannoy3(a - di, b - dj, c - dk)
    return tot


def nw(s, t, sub, gap) -> int:
    """Textbook global pairwise score: H[i][j] = max(diag + sub, up + gap, left + gap)."""
    n, m = len(s), len(t)
    h = np.zeros((n + 1, m + 1), dtype=np.int64)
    for i in range(1, n + 1):
        h[i, 0] = i * gap
    for j in range(1, m + 1):
        h[0, j] = j * gap
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            h[i, j] = max(h[i - 1, j - 1] + int(sub[int(s[i - 1])][int(t[j - 1])]),
                          h[i - 1, j] + gap, h[i, j - 1] + gap)
    return int(h[n, m])


def nw_brute(s, t, sub, gap) -> int:
    """Two-row alignments enumerated explicitly (pins ``nw`` itself)."""
    best = None

    def rec(i, j, acc):
        nonlocal best
        if i == len(s) and j == len(t):
            best = acc if best is None else max(best, acc)
            return
        if i < len(s) and j < len(t):
            rec(i + 1, j + 1, acc + int(sub[int(s[i])][int(t[j])]))
        if i < len(s):
            rec(i + 1, j, acc + gap)
        if j < len(t):
            rec(i, j + 1, acc + gap)

    rec(0, 0, 0)
    return best


def padded_alignment_score(seqs, sub, gap) -> int:
    """SOP score of one explicit alignment: every row padded with trailing gaps."""
    L = max(len(s) for s in seqs)
    if L == 0:
        return 0
    rows = [list(map(int, s)) + [GAP] * (L - len(s)) for s in seqs]
    return sum(column_sop((rows[0][p], rows[1][p], rows[2][p]), sub, gap) for p in range(L))


def random_symmetric_sub(rng, lo=-3, hi=3):
    m = rng.integers(lo, hi + 1, size=(4, 4))
    return np.triu(m) + np.triu(m, 1).T
