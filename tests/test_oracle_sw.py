"""Pins for the scalar Smith-Waterman oracle (CPU only).

The oracle is checked against things other than itself: exhaustive enumeration
of alignments, the cubic general-gap recurrence, closed forms and invariants
that follow from the definition (Section 4: local-alignment score under a
substitution matrix; affine gap model W(k) = go + (k-1)*ge).
"""
import numpy as np
import pytest

import cmgen
from oracle import sw, sw_span, sw_batch, span_batch
from oracle.brute import enumerate_local, general_gap, ungapped_best

M0 = cmgen.make_matrix()
GO, GE = cmgen.GAP_OPEN, cmgen.GAP_EXTEND


def rand_seq(rng, lo, hi, alphabet=20):
    return rng.integers(0, alphabet, size=int(rng.integers(lo, hi + 1))).astype(np.uint8)


def tie_matrix():
    """Residues 0..3: mutual score 0 among 0,1; strong matches elsewhere (tie-heavy)."""
    M = M0.copy()
    M[0, 1] = M[1, 0] = 0
    M[0, 0] = M[1, 1] = 4
    M[2, 3] = M[3, 2] = 0
    return M


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_tiny(seed):
    rng = np.random.default_rng(1000 + seed)
    mats = [M0, tie_matrix()]
    params = [(GO, GE), (-3, -1), (-2, -2), (-4, 0)]
    for trial in range(40):
        M = mats[trial % 2]
        go, ge = params[trial % len(params)]
        alpha = 4 if trial % 3 == 0 else 20       # small alphabet => many matches and ties
        a = rand_seq(rng, 0, 5, alpha)
        b = rand_seq(rng, 0, 5, alpha)
        S, end, start = enumerate_local(a, b, M, go, ge)
        got = sw_span(a, b, M, go, ge)
        assert got[0] == S, (a, b, go, ge)
        assert (got[1], got[2]) == end, (a, b, go, ge)
        assert (got[3], got[4]) == start, (a, b, go, ge)


def test_bruteforce_len6():
    rng = np.random.default_rng(7)
    for _ in range(3):
        a = rng.integers(0, 4, size=6).astype(np.uint8)
        b = rng.integers(0, 4, size=6).astype(np.uint8)
        S, end, start = enumerate_local(a, b, tie_matrix(), -3, -1)
        got = sw_span(a, b, tie_matrix(), -3, -1)
        assert got == (S, end[0], end[1], start[0], start[1])


def test_general_gap_recurrence():
    rng = np.random.default_rng(11)
    params = [(GO, GE), (-5, -2), (-3, -3), (-6, 0)]
    for t in range(30):
        go, ge = params[t % len(params)]
        alpha = 5 if t % 2 else 20
        a = rand_seq(rng, 1, 30, alpha)
        b = rand_seq(rng, 1, 30, alpha)
        assert sw(a, b, M0, go, ge)[0] == general_gap(a, b, M0, go, ge)


def test_general_gap_longer():
    rng = np.random.default_rng(12)
    anc = rng.integers(0, 20, size=60).astype(np.uint8)
    a = cmgen.mutate(rng, anc)
    b = cmgen.mutate(rng, anc)
    assert sw(a, b, M0, GO, GE)[0] == general_gap(a, b, M0, GO, GE)


def test_symmetry_and_transposed_end():
    rng = np.random.default_rng(13)
    for _ in range(40):
        a = rand_seq(rng, 0, 120)
        b = rand_seq(rng, 0, 120)
        s, ei, ej = sw(a, b, M0)
        s2, fi, fj = sw(b, a, M0)
        assert s == s2
        if s > 0:
            # H(a,b) at the transposed end cell of (b,a) must also hold S:
            # the prefix pair a[..fj], b[..fi] reaches S.
            assert sw(a[:fj + 1], b[:fi + 1], M0)[0] == s


def test_reversal():
    rng = np.random.default_rng(14)
    for _ in range(40):
        a = rand_seq(rng, 0, 150)
        b = rand_seq(rng, 0, 150)
        assert sw(a, b, M0)[0] == sw(a[::-1], b[::-1], M0)[0]


def test_self_score_closed_form():
    # diag >= 4 > 3 >= off-diag: the best alignment of a with itself is the identity.
    rng = np.random.default_rng(15)
    assert M0.diagonal().min() >= 4 and (M0 - np.diag(M0.diagonal())).max() <= 3
    for _ in range(20):
        a = rand_seq(rng, 1, 300)
        S, ei, ej, si, sj = sw_span(a, a, M0)
        assert S == int(M0[a, a].sum())
        assert (ei, ej, si, sj) == (len(a) - 1, len(a) - 1, 0, 0)


def test_bound_and_substring():
    rng = np.random.default_rng(16)
    for _ in range(20):
        a = rand_seq(rng, 1, 150)
        b = rand_seq(rng, 1, 150)
        self_a = int(M0[a, a].sum())
        self_b = int(M0[b, b].sum())
        assert sw(a, b, M0)[0] <= min(self_a, self_b)
        x = rand_seq(rng, 0, 40)
        y = rand_seq(rng, 0, 40)
        big = np.concatenate([x, a, y])
        S, ei, ej, si, sj = sw_span(a, big, M0)
        assert S == self_a
        assert (ei, si) == (len(a) - 1, 0)
        # the first exact occurrence of a inside big
        first = next(k for k in range(len(big) - len(a) + 1) if np.array_equal(big[k:k + len(a)], a))
        assert (sj, ej) == (first, first + len(a) - 1)


def test_single_residue():
    rng = np.random.default_rng(17)
    for _ in range(40):
        x = rng.integers(0, 20, size=1).astype(np.uint8)
        b = rand_seq(rng, 0, 60)
        s, ei, ej = sw(x, b, M0)
        vals = [int(M0[x[0], c]) for c in b]
        expect = max([0] + vals)
        assert s == expect
        if expect > 0:
            assert (ei, ej) == (0, vals.index(expect))
        else:
            assert (ei, ej) == (-1, -1)


def test_no_gap_limit_is_kadane():
    rng = np.random.default_rng(18)
    for _ in range(30):
        a = rand_seq(rng, 0, 80)
        b = rand_seq(rng, 0, 80)
        assert sw(a, b, M0, -10**6, -1)[0] == ungapped_best(a, b, M0)


def test_monotone_under_append():
    rng = np.random.default_rng(19)
    for _ in range(30):
        a = rand_seq(rng, 0, 100)
        b = rand_seq(rng, 0, 100)
        s = sw(a, b, M0)[0]
        a2 = np.concatenate([a, rand_seq(rng, 1, 20)])
        b2 = np.concatenate([rand_seq(rng, 1, 20), b])
        assert sw(a2, b, M0)[0] >= s
        assert sw(a, b2, M0)[0] >= s


def test_empty_and_all_zero():
    assert sw(np.zeros(0, np.uint8), np.arange(5, dtype=np.uint8), M0) == (0, -1, -1)
    assert sw(np.zeros(0, np.uint8), np.zeros(0, np.uint8), M0) == (0, -1, -1)
    # every pair scores negative: the empty alignment wins
    M = -np.ones((20, 20), np.int32)
    assert sw_span(np.arange(5, dtype=np.uint8), np.arange(5, dtype=np.uint8), M) == (0, -1, -1, -1, -1)


def test_batch_matches_single():
    ds = cmgen.uniform_pool(30, 0, 200, seed=21)
    rng = np.random.default_rng(22)
    pairs = cmgen.random_pairs(rng, ds.n, 60)
    sc, ea, eb = sw_batch(ds.residues, ds.offsets, pairs, ds.matrix)
    sp = span_batch(ds.residues, ds.offsets, pairs, ds.matrix)
    for p, (x, y) in enumerate(pairs):
        s, ei, ej = sw(ds.seq(x), ds.seq(y), ds.matrix)
        assert (sc[p], ea[p], eb[p]) == (s, ei, ej)
        assert tuple(sp[p, :3]) == (s, ei, ej)


def test_matrix_properties():
    M = cmgen.make_matrix()
    assert M.dtype == np.int32 and M.shape == (20, 20)
    assert np.array_equal(M, M.T)
    d = M.diagonal()
    off = M[~np.eye(20, dtype=bool)]
    assert d.min() >= 4 and d.max() <= 11
    assert off.min() >= -4 and off.max() <= 3
    # expected score of two background residues must be clearly negative
    assert M.mean() <= -1.8


def test_matrix_gate_unrelated_scores():
    """Unrelated sequences must score far below the threshold even when long."""
    rng = np.random.default_rng(23)
    L = 2000
    scores = [sw(rand_seq(rng, L, L), rand_seq(rng, L, L), M0)[0] for _ in range(12)]
    assert max(scores) < 100, scores


def test_family_members_are_similar():
    """Members of one family (length ~350) score well above the threshold."""
    rng = np.random.default_rng(24)
    anc = rng.integers(0, 20, size=350).astype(np.uint8)
    s = [sw(cmgen.mutate(rng, anc), cmgen.mutate(rng, anc), M0)[0] for _ in range(6)]
    assert min(s) > 200, s


# ---- traceback (alignment columns between the start and end cells) ----

def _columns_score(a, b, cols, sa, sb, M, go, ge):
    """Score of an alignment given as columns, summed directly: matrix entries
    of aligned pairs, go + (k-1) ge for every maximal run of k gap columns of
    one kind.  Also returns the end cell reached."""
    i, j, s, prev = sa, sb, 0, None
    for ch in cols:
        if ch == "M":
            s += int(M[a[i], b[j]])
            i += 1
            j += 1
        elif ch == "I":
            s += ge if prev == "I" else go
            i += 1
        else:
            s += ge if prev == "D" else go
            j += 1
        prev = ch
    return s, i - 1, j - 1


def test_traceback_columns_score_and_box():
    """Random related and unrelated pairs: the columns start and end with an
    aligned pair, consume exactly the [start, end] box, and score S."""
    import cmgen
    from oracle import traceback_batch
    rng = np.random.default_rng(301)
    fam = cmgen.family_dataset(6, [4] * 6, lambda r: int(r.integers(30, 300)), 1, 400, 302)
    pairs = cmgen.random_pairs(rng, fam.n, 150)
    for go, ge in ((-11, -1), (-5, -5), (-3, 0)):
        ops, span = traceback_batch(fam.residues, fam.offsets, pairs, fam.matrix, go, ge)
        for (x, y), cols, (S, ea, eb, sa, sb) in zip(pairs, ops, span):
            if S == 0:
                assert cols == ""
                continue
            assert cols[0] == "M" and cols[-1] == "M"
            s, ei, ej = _columns_score(fam.seq(x), fam.seq(y), cols, sa, sb, fam.matrix, go, ge)
            assert (s, ei, ej) == (S, ea, eb)


def _flat_columns(cols):
    n = np.array([len(c) for c in cols], np.int32)
    cap = n + 3                                   # slack: offsets need not be tight
    off = np.zeros(len(cols) + 1, np.int64)
    np.cumsum(cap, out=off[1:])
    ops = np.zeros(max(int(off[-1]), 1), np.uint8)
    for p, c in enumerate(cols):
        ops[off[p]:off[p] + len(c)] = np.frombuffer(c.encode(), np.uint8)
    return ops, off, n


def test_vectorised_column_checker():
    """The batch checker used on full-size GPU output: the oracle's columns
    pass it under several gap models, and planted mistakes (a wrong gap cost,
    a shifted start cell, a first column that is a gap, a swapped interior
    pair of columns, a truncated alignment) are caught in the pairs where they
    were planted and nowhere else."""
    from alignment_columns import check_columns
    from oracle import traceback_batch
    rng = np.random.default_rng(331)
    fam = cmgen.family_dataset(8, [5] * 8, lambda r: int(r.integers(20, 300)), 1, 400, 332)
    pairs = cmgen.random_pairs(rng, fam.n, 400)
    for go, ge in ((-11, -1), (-5, -5), (-3, 0)):
        cols, span = traceback_batch(fam.residues, fam.offsets, pairs, fam.matrix, go, ge)
        ops, off, n = _flat_columns(cols)
        assert check_columns(fam.residues, fam.offsets, pairs, fam.matrix, go, ge, span, ops, off, n) == {}
    gapped = [p for p, c in enumerate(cols) if "II" in c or "DD" in c]
    assert len(gapped) > 20
    # extension cost off by one: exactly the alignments with a gap longer than one column
    bad = check_columns(fam.residues, fam.offsets, pairs, fam.matrix, go, ge - 1, span, ops, off, n)
    assert list(bad) == ["score"] and sorted(bad["score"]) == gapped
    pos = [p for p in range(len(cols)) if span[p, 0] > 0]
    # start cell moved by one row
    sp = span.copy()
    sp[pos[0], 3] += 1
    bad = check_columns(fam.residues, fam.offsets, pairs, fam.matrix, go, ge, sp, ops, off, n)
    assert set(bad) <= {"consumes_a", "score", "inside_sequences"} and list(bad["consumes_a"]) == [pos[0]]
    # a gap as the first column
    c2 = list(cols)
    c2[pos[1]] = "D" + cols[pos[1]][1:]
    o2, f2, n2 = _flat_columns(c2)
    bad = check_columns(fam.residues, fam.offsets, pairs, fam.matrix, go, ge, span, o2, f2, n2)
    assert list(bad["begins_with_M"]) == [pos[1]] and all(set(v) == {pos[1]} for v in bad.values())
    # an interior "MI" swapped to "IM" where the moved residue changes the aligned value
    c3, planted = list(cols), []
    for p in pos:
        k = cols[p].find("MI", 1)
        if k > 0:
            c3[p] = cols[p][:k] + "IM" + cols[p][k + 2:]
            planted.append(p)
    o3, f3, n3 = _flat_columns(c3)
    bad = check_columns(fam.residues, fam.offsets, pairs, fam.matrix, go, ge, span, o3, f3, n3)
    flagged = set().union(*[set(v) for v in bad.values()]) if bad else set()
    assert planted and flagged <= set(planted) and len(flagged) >= len(planted) // 2
    # the last column dropped
    c4 = list(cols)
    c4[pos[2]] = cols[pos[2]][:-1]
    o4, f4, n4 = _flat_columns(c4)
    bad = check_columns(fam.residues, fam.offsets, pairs, fam.matrix, go, ge, span, o4, f4, n4)
    assert all(set(v) == {pos[2]} for v in bad.values()) and "consumes_a" in bad and "consumes_b" in bad
    # a count past its capacity, and columns for a pair whose score is 0
    n5 = n.copy()
    n5[pos[3]] = off[pos[3] + 1] - off[pos[3]] + 1
    sp = span.copy()
    sp[pos[4], 0] = 0
    bad = check_columns(fam.residues, fam.offsets, pairs, fam.matrix, go, ge, sp, ops, off, n5)
    assert sorted(bad) == ["capacity", "count_sign"]
    assert list(bad["capacity"]) == [pos[3]] and list(bad["count_sign"]) == [pos[4]]


def test_traceback_identical_sequences_all_aligned():
    import cmgen
    from oracle import traceback_batch
    rng = np.random.default_rng(303)
    a = rng.integers(0, 20, size=120).astype(np.uint8)
    ds = cmgen.from_list([a, a.copy()])
    ops, span = traceback_batch(ds.residues, ds.offsets, np.array([[0, 1]], np.int32), ds.matrix)
    assert ops[0] == "M" * 120 and tuple(span[0][3:]) == (0, 0)


def _all_alignments(R, C):
    """Every global alignment of an R x C box as a column string."""
    out = []

    def rec(r, c, acc):
        if r == R and c == C:
            out.append("".join(acc))
            return
        if r < R and c < C:
            acc.append("M"); rec(r + 1, c + 1, acc); acc.pop()
        if r < R:
            acc.append("I"); rec(r + 1, c, acc); acc.pop()
        if c < C:
            acc.append("D"); rec(r, c + 1, acc); acc.pop()
    rec(0, 0, [])
    return out


def _preferred(u, v):
    """The walk from the end keeps, at the first column (from the end) where
    two optimal alignments differ, an aligned pair first, then the gap kind of
    the column after it, then the other kind (after an aligned pair: 'I' before
    'D')."""
    ru, rv = u[::-1], v[::-1]
    for k in range(min(len(ru), len(rv))):
        if ru[k] != rv[k]:
            state = ru[k - 1] if k else "M"
            order = {"M": "MID", "I": "MID", "D": "MDI"}[state]
            return u if order.index(ru[k]) < order.index(rv[k]) else v
    return u if len(u) <= len(v) else v


def test_traceback_brute_force_tie_break():
    """Tiny pairs, ties provoked (zero-score residue pairs, repeats): the oracle's
    columns are the optimal alignment of the box chosen by the walk's
    preference among all global alignments of the box."""
    import cmgen
    from oracle import traceback_batch
    M = cmgen.make_matrix().copy()
    M[0, 1] = M[1, 0] = 0
    M[2, 3] = M[3, 2] = 0
    rng = np.random.default_rng(304)
    seqs = [rng.integers(0, 4, size=int(rng.integers(1, 7))).astype(np.uint8) for _ in range(40)]
    seqs += [np.array([5, 5, 0, 5, 5], np.uint8), np.array([5, 5, 5, 5], np.uint8)]
    # repeats around a gap make its position ambiguous (several optimal alignments)
    crafted = [([6, 5, 5, 7], [6, 5, 7]), ([6, 5, 5, 5, 7], [6, 5, 7]), ([6, 8, 8, 7], [6, 8, 7]),
               ([6, 5, 7], [6, 5, 5, 7]), ([6, 5, 5, 7, 9, 9], [6, 5, 7, 9]), ([9, 6, 6, 9], [9, 6, 9, 9]),
               ([6, 5, 5, 7, 8, 8, 9], [6, 5, 7, 8, 9])]
    # a very negative mismatch between cheap gaps: 'I' then 'D' ties 'D' then 'I'
    off = M.astype(np.int64) + 1000 * np.eye(20, dtype=np.int64)
    u, v = (int(t) for t in np.unravel_index(np.argmin(off[4:, 4:]), (16, 16)))
    u, v = u + 4, v + 4
    crafted += [([6, u, 7], [6, v, 7]), ([6, u, u, 7], [6, v, v, 7]), ([9, u, 9, 9], [9, v, 9, 9])]
    base = len(seqs)
    for u, v in crafted:
        seqs += [np.array(u, np.uint8), np.array(v, np.uint8)]
    ds = cmgen.from_list(seqs, M)
    pairs = cmgen.random_pairs(rng, ds.n, 300)
    extra = [(base + 2 * k, base + 2 * k + 1) for k in range(len(crafted))]
    pairs = np.concatenate([pairs, np.array(extra + [(y, x) for x, y in extra], np.int32)])
    checked = 0
    several = 0
    for go, ge in ((-11, -1), (-2, -1), (-3, -3), (-1, -1)):
        ops, span = traceback_batch(ds.residues, ds.offsets, pairs, M, go, ge)
        for (x, y), cols, (S, ea, eb, sa, sb) in zip(pairs, ops, span):
            if S == 0:
                continue
            a, b = ds.seq(x), ds.seq(y)
            best, n_opt = None, 0
            for cand in _all_alignments(ea - sa + 1, eb - sb + 1):
                if cand[0] != "M" or cand[-1] != "M":
                    continue
                s, _, _ = _columns_score(a, b, cand, sa, sb, M, go, ge)
                assert s <= S
                if s == S:
                    n_opt += 1
                    best = cand if best is None else _preferred(best, cand)
            assert best == cols, (x, y, go, ge, cols, best)
            checked += 1
            several += n_opt > 1
    assert checked > 200 and several >= 10
