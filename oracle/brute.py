"""Independent checks for the scalar oracle.  Test infrastructure only.

* ``enumerate_local`` lists EVERY local alignment of two short sequences as a
  column sequence and scores it from the definition (sum of substitution
  values plus W(k) = go + (k-1)*ge for each maximal run of k gap columns of one
  kind).  It shares nothing with the dynamic programme.
* ``general_gap`` is the cubic Waterman-Smith-Beyer recurrence, in which a gap
  of any length k is charged W(k) in one step.
* ``ungapped_best`` is the maximum-subarray (Kadane) scan along every
  diagonal, which is the local score when gaps are prohibitively expensive.
"""
from __future__ import annotations

import numpy as np


def enumerate_local(a, b, M, go, ge):
    """(S, end, start) by brute force.

    S is the best score over all alignments of all substring pairs (0 for the
    empty alignment).  ``end`` is the lexicographically smallest last cell
    (i, j) among alignments scoring S, ``start`` the lexicographically largest
    first cell among optimal alignments ending there.  Both are (-1, -1) when
    S == 0.  Alignments are walked depth-first: each step appends one column,
    a pair (i, j), a gap in b (i, -) or a gap in a (-, j).
    """
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    m, n = len(a), len(b)
    best = [0, None, None]   # score, end, start

    def visit(score, i, j, start, last_kind):
        # the alignment so far consumed a[start_i..i-1], b[start_j..j-1]
        if last_kind is not None:
            end = (i - 1, j - 1)
            if score > best[0]:
                best[0], best[1], best[2] = score, end, start
            elif score == best[0] and best[0] > 0:
                if end < best[1] or (end == best[1] and start > best[2]):
                    best[1], best[2] = end, start
        if i < m and j < n:     # aligned pair
            visit(score + M[a[i]][b[j]], i + 1, j + 1, start, "P")
        if i < m:               # gap in b: consumes a[i]
            visit(score + (ge if last_kind == "D" else go), i + 1, j, start, "D")
        if j < n:               # gap in a: consumes b[j]
            visit(score + (ge if last_kind == "I" else go), i, j + 1, start, "I")

    for i0 in range(m + 1):
        for j0 in range(n + 1):
            # An alignment starting with a gap column is also enumerated; its
            # first cell is taken as (i0, j0) like any other.
            visit(0, i0, j0, (i0, j0), None)
    if best[0] == 0:
        return 0, (-1, -1), (-1, -1)
    return best[0], best[1], best[2]


def general_gap(a, b, M, go, ge):
    """Cubic recurrence with gap cost W(k) = go + (k-1)*ge applied per run."""
    m, n = len(a), len(b)
    H = np.zeros((m + 1, n + 1), dtype=np.int64)
    best = 0
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            v = H[i - 1, j - 1] + int(M[a[i - 1]][b[j - 1]])
            for k in range(1, j + 1):
                v = max(v, H[i, j - k] + go + (k - 1) * ge)
            for k in range(1, i + 1):
                v = max(v, H[i - k, j] + go + (k - 1) * ge)
            H[i, j] = max(0, v)
            best = max(best, H[i, j])
    return int(best)


def ungapped_best(a, b, M):
    """Best ungapped local score: maximum subarray along every diagonal."""
    m, n = len(a), len(b)
    best = 0
    for d in range(-(m - 1), n):
        run = 0
        i = max(0, -d)
        j = i + d
        while i < m and j < n:
            run = max(0, run + int(M[a[i]][b[j]]))
            best = max(best, run)
            i += 1
            j += 1
    return best
