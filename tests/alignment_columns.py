"""Checks that hold for alignment columns of any batch, at any size, vectorised
over the batch so that they can cover every pair of a full-size run.

For a pair with Smith-Waterman score S > 0 and start/end cells (sa, sb), (ea,
eb), its columns must be a global alignment of a[sa..ea] with b[sb..eb] (the
'M' and 'I' columns consume a, the 'M' and 'D' columns consume b, each exactly
once, in order), begin and end with an aligned pair, and score exactly S under
the Gotoh model of Section 4 (a substitution value per 'M'; a run of k gap
columns of one kind costs go + (k - 1) * ge, and a run of the other kind that
follows directly opens a new gap).  An alignment of the box that reaches S is
an optimal local alignment, since S is the maximum over all of them.  Which of
several optimal alignments is chosen is not checked here (the oracle's columns
fix that on a sample).
"""
import numpy as np

_M, _I, _D = ord("M"), ord("I"), ord("D")


def check_columns(residues, offsets, pairs, M, go, ge, span, ops, op_off, n_ops):
    """span: [n][5] rows (score, end_a, end_b, start_a, start_b); ops: the byte
    buffer; op_off: [n + 1] offsets into ops (absolute, so a slice of a larger
    batch's offsets works); n_ops: [n] column counts.  Returns a dict from the
    name of each failed property to the indices (into this batch) of the pairs
    that fail it; empty when every pair passes."""
    res = np.asarray(residues, np.uint8)
    off = np.asarray(offsets, np.int64)
    pr = np.asarray(pairs, np.int64).reshape(-1, 2)
    span = np.asarray(span, np.int64).reshape(-1, 5)
    ops = np.asarray(ops, np.uint8)
    op_off = np.asarray(op_off, np.int64)
    n_ops = np.asarray(n_ops, np.int64)
    M = np.asarray(M, np.int64)
    P = len(pr)
    sc, ea, eb, sa, sb = (span[:, k] for k in range(5))
    bad = {}

    def fail(name, mask):
        idx = np.flatnonzero(mask)
        if len(idx):
            bad[name] = idx

    fail("count_sign", np.where(sc > 0, n_ops <= 0, n_ops != 0))
    n = np.where((sc > 0) & (n_ops > 0), n_ops, 0)
    fail("capacity", (n > 0) & (op_off[:-1] + n > op_off[1:]))
    n = np.where(op_off[:-1] + n > op_off[1:], 0, n)
    tot = int(n.sum())
    if tot == 0:
        return bad
    first = np.cumsum(n) - n                      # each pair's first column in the flat arrays
    pid = np.repeat(np.arange(P), n)
    pos = np.arange(tot) - first[pid]
    c = ops[op_off[:-1][pid] + pos]
    isM, isI, isD = c == _M, c == _I, c == _D
    fail("alphabet", np.bincount(pid, ~(isM | isI | isD), minlength=P) > 0)
    has = n > 0
    fail("begins_with_M", has & (ops[np.where(has, op_off[:-1], 0)] != _M))
    fail("ends_with_M", has & (ops[np.where(has, op_off[:-1] + n - 1, 0)] != _M))
    ca = (isM | isI).astype(np.int64)
    cb = (isM | isD).astype(np.int64)
    na = np.bincount(pid, ca, minlength=P).astype(np.int64)
    nb = np.bincount(pid, cb, minlength=P).astype(np.int64)
    fail("consumes_a", has & (na != ea - sa + 1))
    fail("consumes_b", has & (nb != eb - sb + 1))
    # row and column of every 'M': cells consumed before it within its pair
    xa = np.cumsum(ca) - ca
    xb = np.cumsum(cb) - cb
    ai = sa[pid] + (xa - xa[first[pid]])
    bj = sb[pid] + (xb - xb[first[pid]])
    la = off[pr[:, 0] + 1] - off[pr[:, 0]]
    lb = off[pr[:, 1] + 1] - off[pr[:, 1]]
    inside = (ai >= 0) & (ai < la[pid]) & (bj >= 0) & (bj < lb[pid])
    fail("inside_sequences", np.bincount(pid, isM & ~inside, minlength=P) > 0)
    ra = res[off[pr[pid, 0]] + np.clip(ai, 0, la[pid] - 1)]
    rb = res[off[pr[pid, 1]] + np.clip(bj, 0, lb[pid] - 1)]
    prev_same = np.zeros(tot, bool)
    prev_same[1:] = (c[1:] == c[:-1]) & (pos[1:] > 0)
    val = np.where(isM, M[ra, rb], np.where(prev_same, ge, go))
    score = np.bincount(pid, val.astype(np.float64), minlength=P).round().astype(np.int64)
    fail("score", has & (score != sc))
    return bad
