"""Pins for the sequential ClusterMerge oracle (CPU only).

Algorithm 2's FIFO tree shape is checked by hand for small n; Algorithm 1 is
checked against the consequences the paper states in Sections 3.3-3.4: a
transitivity function that never holds forces every pair of elements to meet
once as representatives (the worst case, n(n-1)/2 comparisons); a complete
transitivity function (an equivalence relation) loses no similar pair; and
identical proteins collapse into one cluster after n-1 comparisons.
"""
import numpy as np

import cmgen
from oracle import clustermerge as cm
from oracle import sw


def test_fifo_tree_shape_by_hand():
    assert cm.merge_schedule(1) == []
    assert cm.merge_schedule(2) == [(0, 1, 2)]
    assert cm.merge_schedule(3) == [(0, 1, 3), (2, 3, 4)]
    assert cm.merge_schedule(4) == [(0, 1, 4), (2, 3, 5), (4, 5, 6)]
    # n=5: (0,1)->A, (2,3)->B, (4,A)->C, (B,C)->D
    assert cm.merge_schedule(5) == [(0, 1, 5), (2, 3, 6), (4, 5, 7), (6, 7, 8)]
    assert cm.merge_schedule(6) == [(0, 1, 6), (2, 3, 7), (4, 5, 8), (6, 7, 9), (8, 9, 10)]
    assert cm.merge_schedule(7) == [(0, 1, 7), (2, 3, 8), (4, 5, 9), (6, 7, 10), (8, 9, 11),
                                    (10, 11, 12)]
    assert cm.merge_schedule(8)[-1] == (12, 13, 14)
    assert cm.merge_schedule(9) == [(0, 1, 9), (2, 3, 10), (4, 5, 11), (6, 7, 12), (8, 9, 13),
                                    (10, 11, 14), (12, 13, 15), (14, 15, 16)]
    for n in range(1, 40):
        assert len(cm.merge_schedule(n)) == max(0, n - 1)


def test_never_transitive_is_all_vs_all():
    for n in (1, 2, 5, 9, 17):
        judge = cm.TableJudge(lambda x, y: True, lambda r, s: False)
        clusters, st = cm.bottom_up_merge(n, judge)
        assert st.rep_comparisons == n * (n - 1) // 2
        assert sorted(c.rep for c in clusters) == list(range(n))
        found = {(x, y) for x, y in cm.cluster_pairs(clusters)}
        assert found == {(x, y) for x in range(n) for y in range(x + 1, n)}


def test_equivalence_relation_gives_label_classes():
    rng = np.random.default_rng(3)
    for n in (7, 20, 33):
        lab = rng.integers(0, 4, size=n)
        same = lambda x, y: lab[x] == lab[y]  # noqa: E731
        clusters, st = cm.bottom_up_merge(n, cm.TableJudge(same, same))
        got = sorted(sorted(c.objs) for c in clusters)
        want = sorted(sorted(np.flatnonzero(lab == v).tolist()) for v in np.unique(lab))
        assert got == want
        truth = {(x, y) for x in range(n) for y in range(x + 1, n) if lab[x] == lab[y]}
        assert set(cm.cluster_pairs(clusters)) == truth


def test_identical_proteins_collapse():
    rng = np.random.default_rng(4)
    a = rng.integers(0, 20, size=60).astype(np.uint8)
    ds = cmgen.from_list([a] * 4)
    clusters, pairs, st = cm.clustermerge(ds.residues, ds.offsets, ds.matrix)
    assert len(clusters) == 1
    assert clusters[0].rep == 3 and clusters[0].objs == [3, 2, 1, 0]
    assert st.rep_comparisons == 3
    assert [(x, y) for x, y, _ in pairs] == [(x, y) for x in range(4) for y in range(x + 1, 4)]


def test_exchange_semantics():
    # reps 0 and 2 similar but never transitive; member 1 of cluster(0) is
    # similar to rep 2, member 3 of cluster(2) is not similar to rep 0.
    sim = {(0, 1), (2, 3), (0, 2), (1, 2)}
    similar = lambda x, y: (min(x, y), max(x, y)) in sim  # noqa: E731
    trans_within = {(0, 1), (2, 3)}   # absorber, absorbed
    transitive = lambda r, s: (r, s) in trans_within or (s, r) in trans_within  # noqa: E731
    clusters, st = cm.bottom_up_merge(4, cm.TableJudge(similar, transitive))
    byrep = {c.rep: c.objs for c in clusters}
    # (0,1): cluster(1) absorbs cluster(0) -> rep 1, objs [1, 0]
    # (2,3): cluster(3) absorbs cluster(2) -> rep 3, objs [3, 2]
    # merge reps 1 and 3: not similar -> unchanged
    assert byrep == {1: [1, 0], 3: [3, 2]}


def test_exchange_adds_reps_and_similar_members():
    sim = {(0, 2), (1, 2), (0, 3)}
    similar = lambda x, y: (min(x, y), max(x, y)) in sim  # noqa: E731
    never = lambda r, s: False  # noqa: E731
    # Tree: (0,1) -> [c0, c1]; (2,3) -> [c2, c3]; then merge the two sets.
    clusters, st = cm.bottom_up_merge(4, cm.TableJudge(similar, never))
    byrep = {c.rep: c.objs for c in clusters}
    assert byrep == {0: [0, 2, 3], 1: [1, 2], 2: [2, 0, 1], 3: [3, 0]}


def test_precision_and_recall_small_families():
    ds = cmgen.allvsall_small()
    clusters, found, st = cm.clustermerge(ds.residues, ds.offsets, ds.matrix)
    truth = cm.allvsall(ds.residues, ds.offsets, ds.matrix)
    tset = {(x, y) for x, y, _ in truth}
    # precision is 100% by construction: every reported pair was aligned
    assert all((x, y) in tset for x, y, _ in found)
    for x, y, s in found[:50]:
        assert sw(ds.seq(x), ds.seq(y), ds.matrix)[0] == s
    r = cm.recall(found, truth)
    assert r >= 0.9, r
    assert st.rep_comparisons < ds.n * (ds.n - 1) // 2
    # every element ends in at least one cluster; reps are members of their own cluster
    members = set()
    for c in clusters:
        assert c.rep in c.objs and len(set(c.objs)) == len(c.objs)
        members.update(c.objs)
    assert members == set(range(ds.n))


def test_screened_replay_special_cases():
    """A screen that keeps everything, or a size guard every pair passes, is plain
    ClusterMerge; a screen that drops every representative pair leaves singletons."""
    ds = cmgen.allvsall_small()
    ref_c, ref_p, ref_s = cm.clustermerge(ds.residues, ds.offsets, ds.matrix)

    def same(c, p, s):
        assert [(x.rep, x.objs) for x in c] == [(x.rep, x.objs) for x in ref_c]
        assert p == ref_p and s == ref_s

    same(*cm.clustermerge_screened(ds.residues, ds.offsets, ds.matrix, lambda x, y: True, 7))
    never = lambda x, y: False  # noqa: E731
    same(*cm.clustermerge_screened(ds.residues, ds.offsets, ds.matrix, never, cm.STAGE_REP, min_product=1))
    for mp in (0, 2):   # every merge starts from singletons, so a guard of 2 never fires
        c, p, s = cm.clustermerge_screened(ds.residues, ds.offsets, ds.matrix, never, cm.STAGE_REP,
                                           min_product=mp)
        assert len(c) == ds.n and p == [] and s.full_merges == 0 and s.exchanges == 0
        assert s.rep_comparisons == ds.n * (ds.n - 1) // 2


def test_generator_divergence_parameter():
    """The family generator's member divergence: the defaults are the workload's
    rates (0.30 substitutions, 0.05 indel events per position); a different
    substitution rate keeps the lengths (same indel draws) and changes the
    fraction of positions that differ from a zero-divergence copy."""
    base = cmgen.family_dataset(4, [5] * 4, lambda r: 300, 30, 2000, 17)
    same = cmgen.family_dataset(4, [5] * 4, lambda r: 300, 30, 2000, 17, sub_rate=0.30, indel_rate=0.05)
    assert np.array_equal(base.residues, same.residues) and np.array_equal(base.offsets, same.offsets)
    none = cmgen.family_dataset(4, [5] * 4, lambda r: 300, 30, 2000, 17, sub_rate=0.0, indel_rate=0.0)
    half = cmgen.family_dataset(4, [5] * 4, lambda r: 300, 30, 2000, 17, sub_rate=0.5, indel_rate=0.0)
    assert np.array_equal(none.offsets, half.offsets)
    diff = (none.residues != half.residues).mean()
    assert 0.45 < diff < 0.55
    lo = cmgen.family_dataset(4, [5] * 4, lambda r: 300, 30, 2000, 17, sub_rate=0.2)
    assert np.array_equal(lo.offsets, base.offsets) and not np.array_equal(lo.residues, base.residues)


def _as_prev(clusters):
    return [(c.rep, list(c.objs)) for c in clusters]


def test_extend_from_nothing_is_clustermerge():
    """With no previous elements, incremental classification is ClusterMerge."""
    ds = cmgen.clustermerge_families(n_seqs=40, n_families=6, seed=221, median=90, hi=200)
    c1, p1, s1 = cm.clustermerge(ds.residues, ds.offsets, ds.matrix)
    c2, p2, s2 = cm.clustermerge_extend(ds.residues, ds.offsets, ds.matrix, [], 0)
    assert _as_prev(c1) == _as_prev(c2) and p1 == p2
    assert (s1.rep_comparisons, s1.exchange_alignments, s1.full_merges, s1.exchanges) == \
           (s2.rep_comparisons, s2.exchange_alignments, s2.full_merges, s2.exchanges)


def test_extend_without_new_elements_keeps_the_clustering():
    ds = cmgen.clustermerge_families(n_seqs=40, n_families=6, seed=222, median=90, hi=200)
    c1, p1, _ = cm.clustermerge(ds.residues, ds.offsets, ds.matrix)
    c2, p2, s2 = cm.clustermerge_extend(ds.residues, ds.offsets, ds.matrix, _as_prev(c1), ds.n)
    assert _as_prev(c2) == _as_prev(c1) and p2 == p1 and s2.rep_comparisons == 0


def test_extend_with_a_copy_of_a_representative():
    """A new protein identical to a representative covers it completely with a
    score far above mT, so the new singleton absorbs that representative's
    cluster (the second set's cluster is tested as absorber first) and becomes
    its representative; the number of clusters is unchanged."""
    ds = cmgen.clustermerge_families(n_seqs=30, n_families=5, seed=223, median=150, hi=300)
    c1, _, _ = cm.clustermerge(ds.residues, ds.offsets, ds.matrix)
    big = max(c1, key=lambda c: len(c.objs))
    copy = ds.seq(big.rep).copy()
    d2 = cmgen.from_list([ds.seq(i) for i in range(ds.n)] + [copy], ds.matrix)
    c2, _, s2 = cm.clustermerge_extend(d2.residues, d2.offsets, d2.matrix, _as_prev(c1), ds.n)
    assert len(c2) == len(c1)
    mine = [c for c in c2 if c.rep == ds.n]
    assert len(mine) == 1 and mine[0].objs == [ds.n] + big.objs
    assert s2.full_merges >= 1


def test_extend_never_transitive_compares_every_pair_once():
    """mT out of reach: no full merge, so every new element meets every other
    new element and every previous cluster exactly once as representatives."""
    ds = cmgen.clustermerge_families(n_seqs=36, n_families=6, seed=224, median=80, hi=160)
    n_prev = 24
    c1, _, _ = cm.clustermerge(ds.residues[: ds.offsets[n_prev]], ds.offsets[: n_prev + 1], ds.matrix, mT=10**6)
    assert len(c1) == n_prev
    c2, pairs, s2 = cm.clustermerge_extend(ds.residues, ds.offsets, ds.matrix, _as_prev(c1), n_prev, mT=10**6)
    n_new = ds.n - n_prev
    assert s2.rep_comparisons == n_new * (n_new - 1) // 2 + n_prev * n_new
    assert s2.full_merges == 0 and len(c2) == ds.n


# ---------------------------------------------------------------------------
# Section 4's transitivity test, pinned on asymmetric pairs.  A short protein A
# that occurs whole inside a longer protein D (with long flanks that A does not
# cover) is nearly covered by the alignment, D is not: D's cluster may stand
# for A's (absorb it), never the other way round, whichever set each one
# starts in.  The comparators are strict: score > mT and uncovered < mU.
# ---------------------------------------------------------------------------
def _embedded_pair(seed=31, core=60, flank=100):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 20, size=core).astype(np.uint8)
    d = np.concatenate([rng.integers(0, 20, size=flank), a, rng.integers(0, 20, size=flank)]).astype(np.uint8)
    return a, d


def test_longer_protein_absorbs_the_embedded_one_in_either_set_order():
    a, d = _embedded_pair()
    M = cmgen.make_matrix()
    # the local alignment of A inside D is A against itself: S(A, D) = S(A, A),
    # all of A covered and both flanks of D left over
    s_aa = sw(a, a, M)[0]
    from oracle import sw_span
    S, ei, ej, si, sj = sw_span(a, d, M)
    assert S == s_aa == int(sum(M[x, x] for x in a)) and S > 166
    assert (si, ei) == (0, len(a) - 1) and (sj, ej) == (100, 100 + len(a) - 1)

    # A is element 0 (first set), D element 1 (second set): the second set's
    # cluster (D) absorbs the first (A)
    ds = cmgen.from_list([a, d], M)
    clusters, pairs, st = cm.clustermerge(ds.residues, ds.offsets, ds.matrix)
    assert [(c.rep, c.objs) for c in clusters] == [(1, [1, 0])]
    assert st.full_merges == 1 and st.exchanges == 0 and pairs == [(0, 1, S)]

    # D is element 0 (first set), A element 1: D's cluster, now in the first
    # set, absorbs A's and keeps its place; A's cluster never absorbs D
    ds = cmgen.from_list([d, a], M)
    clusters, pairs, st = cm.clustermerge(ds.residues, ds.offsets, ds.matrix)
    assert [(c.rep, c.objs) for c in clusters] == [(0, [0, 1])]
    assert st.full_merges == 1 and st.exchanges == 0 and pairs == [(0, 1, S)]

    # the judge's answers themselves, both orientations
    for order, (r1, r2) in ((("a", "d"), (0, 1)), (("d", "a"), (0, 1))):
        seqs = {"a": a, "d": d}
        ds = cmgen.from_list([seqs[order[0]], seqs[order[1]]], M)
        judge = cm.ProteinJudge(ds.residues, ds.offsets, ds.matrix)
        similar, c2_takes_c1, c1_takes_c2 = judge.rep_test(r1, r2)
        assert similar
        # the cluster whose representative is D is the absorber
        assert c2_takes_c1 == (order[1] == "d") and c1_takes_c2 == (order[0] == "d")


def test_score_equal_to_mT_is_not_transitive():
    a, d = _embedded_pair(seed=32)
    M = cmgen.make_matrix()
    S = sw(a, d, M)[0]
    ds = cmgen.from_list([a, d], M)
    # score == mT: not "above" mT, so the similar representatives exchange
    # members instead (each cluster receives the other, since both are similar)
    clusters, pairs, st = cm.clustermerge(ds.residues, ds.offsets, ds.matrix, mT=S)
    assert st.full_merges == 0 and st.exchanges == 1
    assert [(c.rep, c.objs) for c in clusters] == [(0, [0, 1]), (1, [1, 0])]
    assert pairs == [(0, 1, S)]
    # one below: the full merge happens
    clusters, _, st = cm.clustermerge(ds.residues, ds.offsets, ds.matrix, mT=S - 1)
    assert st.full_merges == 1 and [(c.rep, c.objs) for c in clusters] == [(1, [1, 0])]


def test_uncovered_equal_to_mU_is_not_transitive():
    """A carries a few residues before the part it shares with D; the count of
    its residues outside the alignment decides: equal to mU is not fewer."""
    rng = np.random.default_rng(33)
    core = rng.integers(0, 20, size=70).astype(np.uint8)
    # a prefix that scores badly against D's flank (residue 0 repeated, D's
    # flank drawn without residue 0) so the alignment cannot extend into it
    a = np.concatenate([np.zeros(9, np.uint8), core])
    flank_l = rng.integers(1, 20, size=120).astype(np.uint8)
    flank_r = rng.integers(1, 20, size=120).astype(np.uint8)
    d = np.concatenate([flank_l, core, flank_r])
    M = cmgen.make_matrix()
    from oracle import sw_span
    S, ei, ej, si, sj = sw_span(a, d, M)
    u_a = len(a) - (ei - si + 1)
    u_d = len(d) - (ej - sj + 1)
    assert S > 166 and 0 < u_a < u_d and u_d >= 200
    ds = cmgen.from_list([a, d], M)
    for mU, merged in ((u_a, False), (u_a + 1, True)):
        clusters, pairs, st = cm.clustermerge(ds.residues, ds.offsets, ds.matrix, mU=mU)
        assert st.full_merges == (1 if merged else 0), (mU, u_a)
        want = [(1, [1, 0])] if merged else [(0, [0, 1]), (1, [1, 0])]
        assert [(c.rep, c.objs) for c in clusters] == want
        assert pairs == [(0, 1, S)]


def test_score_equal_to_T_is_similar():
    """Similarity is score >= T (Algorithm 1 skips a pair only below T)."""
    rng = np.random.default_rng(34)
    x = rng.integers(0, 20, size=80).astype(np.uint8)
    y = x.copy()
    y[::3] = rng.integers(0, 20, size=len(y[::3]))
    M = cmgen.make_matrix()
    S = sw(x, y, M)[0]
    assert S > 30
    ds = cmgen.from_list([x, y], M)
    never = 10 ** 6
    for T, found in ((S, True), (S + 1, False)):
        clusters, pairs, st = cm.clustermerge(ds.residues, ds.offsets, ds.matrix, T=T, mT=never)
        assert st.rep_comparisons == 1 and st.full_merges == 0
        assert st.exchanges == (1 if found else 0)
        assert pairs == ([(0, 1, S)] if found else [])
