"""ClusterMerge written out sequentially.  Test infrastructure only.

Algorithm 2 (BottomUpMerge, Section 3.2): every element starts as a one-cluster
set in a FIFO queue; two sets are popped, merged with Algorithm 1 and the
result is pushed back until one set remains.

Algorithm 1 (Cluster Set Merge, Section 3.1): every cluster of the first set is
compared with every not-yet-merged cluster of the second set through their
representatives.  Similar representatives are then tested for transitivity
both ways (Section 3.3: approximate transitivity is not symmetric).  A
transitive pair is fully merged; a similar but non-transitive pair exchanges
members similar to the other representative; dissimilar pairs are left alone.

Section 4 defines the protein transitivity: the score must exceed mT and the
absorbed representative may leave fewer than mU residues outside the local
alignment.

Readings where the paper is silent (each is listed in the design notes):
  * similarity is ``score >= T`` (the listing's "skip if s < T");
  * alignment orientation for representatives: rows = cluster of the first
    set, columns = cluster of the second set;
  * "uncovered" = residues of the absorbed representative outside
    [start, end] on both flanks, from the tie-broken span;
  * ExchangeSimilar takes snapshots of both member lists, adds (in member
    order) the members of the other cluster that are similar to this
    cluster's representative and not already present;
  * a full merge appends the absorbed members in order, skipping any already
    present.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field

import numpy as np

from .sw import sw, sw_span


@dataclass
class Cluster:
    rep: int
    objs: list = field(default_factory=list)
    merged: bool = False


@dataclass
class Stats:
    rep_comparisons: int = 0       # f(rep1, rep2) evaluations of Algorithm 1
    exchange_alignments: int = 0   # member-vs-representative evaluations
    full_merges: int = 0
    exchanges: int = 0


def merge_schedule(n: int):
    """The FIFO merge order of Algorithm 2 as (first, second, result) set ids.

    Sets 0..n-1 are the singletons in element order; merges create n, n+1, ...
    """
    q = deque(range(n))
    out, nxt = [], n
    while len(q) > 1:
        x = q.popleft()
        y = q.popleft()
        out.append((x, y, nxt))
        q.append(nxt)
        nxt += 1
    return out


class ProteinJudge:
    """f = Smith-Waterman score; R = score > mT and absorbed rep's uncovered < mU."""

    def __init__(self, residues, offsets, M, T=120, mT=166, mU=15, go=-11, ge=-1):
        self.res = np.asarray(residues, dtype=np.uint8)
        self.off = np.asarray(offsets, dtype=np.int64)
        self.M = np.asarray(M, dtype=np.int32)
        self.T, self.mT, self.mU, self.go, self.ge = T, mT, mU, go, ge
        self._score = {}
        self._span = {}

    def seq(self, i):
        return self.res[self.off[i]:self.off[i + 1]]

    def score(self, x, y):
        key = (x, y) if x <= y else (y, x)
        s = self._score.get(key)
        if s is None:
            s = sw(self.seq(key[0]), self.seq(key[1]), self.M, self.go, self.ge)[0]
            self._score[key] = s
        return s

    def rep_test(self, r1, r2):
        """(similar, cluster2 absorbs cluster1, cluster1 absorbs cluster2) for reps r1 (set 1), r2 (set 2)."""
        key = (r1, r2)
        v = self._span.get(key)
        if v is None:
            s = self.score(r1, r2)
            if s > self.mT:
                S, ei, ej, si, sj = sw_span(self.seq(r1), self.seq(r2), self.M, self.go, self.ge)
                assert S == s
                u1 = len(self.seq(r1)) - (ei - si + 1)
                u2 = len(self.seq(r2)) - (ej - sj + 1)
                v = (s >= self.T, u1 < self.mU, u2 < self.mU)
            else:
                v = (s >= self.T, False, False)
            self._span[key] = v
        return v

    def member_similar(self, m, rep):
        return self.score(m, rep) >= self.T


class TableJudge:
    """Injected similarity and transitivity (for the tree-shape and semantic pins)."""

    def __init__(self, similar, transitive):
        self._similar = similar          # (x, y) -> bool
        self._transitive = transitive    # (absorber, absorbed) -> bool

    def rep_test(self, r1, r2):
        s = self._similar(r1, r2)
        return (s, s and self._transitive(r2, r1), s and self._transitive(r1, r2))

    def member_similar(self, m, rep):
        return self._similar(m, rep)


def _append_missing(dst, src):
    have = set(dst)
    for x in src:
        if x not in have:
            dst.append(x)
            have.add(x)


def exchange_similar(c1, c2, judge, stats):
    m1 = list(c1.objs)
    m2 = list(c2.objs)
    in1, in2 = set(m1), set(m2)
    add1 = [m for m in m2 if m not in in1 and judge.member_similar(m, c1.rep)]
    add2 = [m for m in m1 if m not in in2 and judge.member_similar(m, c2.rep)]
    stats.exchange_alignments += sum(1 for m in m2 if m not in in1)
    stats.exchange_alignments += sum(1 for m in m1 if m not in in2)
    c1.objs.extend(add1)
    c2.objs.extend(add2)
    stats.exchanges += 1


# How two live clusters relate, from their representatives (Section 3.1: the
# similarity f >= T; Section 4: the transitivity test that lets one cluster
# absorb the other; approximate transitivity is not symmetric, Section 3.3).
APART, INTO_SECOND, INTO_FIRST, EXCHANGE = range(4)


def relation(c1, c2, judge, stats):
    """Relation of cluster c1 (first set) to cluster c2 (second set)."""
    stats.rep_comparisons += 1
    similar, second_absorbs_first, first_absorbs_second = judge.rep_test(c1.rep, c2.rep)
    if not similar:
        return APART
    if second_absorbs_first:
        return INTO_SECOND
    return INTO_FIRST if first_absorbs_second else EXCHANGE


def absorb(keeper, gone, stats):
    """Full merge: the absorbed cluster's members join the keeper (in order,
    skipping members already present) and the absorbed cluster is retired."""
    _append_missing(keeper.objs, gone.objs)
    gone.merged = True
    stats.full_merges += 1


def sweep_row(c1, cs2, judge, stats):
    """Compare c1 with the second set's clusters that are still live, in set
    order.  Returns True when c1 was absorbed, which ends its comparisons."""
    for c2 in (c for c in cs2 if not c.merged):     # liveness read as the row advances
        rel = relation(c1, c2, judge, stats)
        if rel == INTO_SECOND:
            absorb(c2, c1, stats)
            return True
        if rel == INTO_FIRST:
            absorb(c1, c2, stats)
        elif rel == EXCHANGE:
            exchange_similar(c1, c2, judge, stats)
    return False


def merge(cs1, cs2, judge, stats):
    """Algorithm 1 (Section 3.1) on two ordered cluster lists: every cluster of
    the first set, in order, is swept against the second set; the new list is
    the first set's surviving clusters followed by the second set's."""
    if hasattr(judge, "begin_merge"):
        judge.begin_merge(cs1, cs2)
    survivors = [c1 for c1 in cs1 if not sweep_row(c1, cs2, judge, stats)]
    return survivors + [c2 for c2 in cs2 if not c2.merged]


def bottom_up_merge(n, judge, stats=None):
    """Algorithm 2 (Section 3.2) over elements 0..n-1 in index order: the sets
    are merged in the FIFO order of merge_schedule; returns (clusters, stats)."""
    stats = stats or Stats()
    sets = {e: [Cluster(e, [e])] for e in range(n)}
    for first, second, result in merge_schedule(n):
        sets[result] = merge(sets.pop(first), sets.pop(second), judge, stats)
    final = next(iter(sets.values())) if sets else []
    return final, stats


def cluster_pairs(clusters):
    """Unique (x, y), x < y, over the members of every final cluster, sorted."""
    s = set()
    for c in clusters:
        objs = sorted(set(c.objs))
        for i in range(len(objs)):
            for j in range(i + 1, len(objs)):
                s.add((objs[i], objs[j]))
    return sorted(s)


def similar_pairs(clusters, score, T):
    """Final stage (Section 6.1): align all pairs inside each cluster, keep score >= T."""
    out = []
    for x, y in cluster_pairs(clusters):
        s = score(x, y)
        if s >= T:
            out.append((x, y, s))
    return out


def clustermerge(residues, offsets, M, T=120, mT=166, mU=15, go=-11, ge=-1):
    """Plain ClusterMerge end to end: (clusters, similar pairs, stats)."""
    n = len(offsets) - 1
    judge = ProteinJudge(residues, offsets, M, T, mT, mU, go, ge)
    clusters, stats = bottom_up_merge(n, judge)
    pairs = similar_pairs(clusters, judge.score, T)
    return clusters, pairs, stats


def clustermerge_extend(residues, offsets, M, prev, n_prev, T=120, mT=166, mU=15, go=-11, ge=-1):
    """Incremental classification of new elements against an existing
    clustering (the concluding remark of the paper: new sequences classified
    against the clusters already formed).  Reading: elements 0..n_prev-1 are
    clustered by `prev` (a list of (rep, members), e.g. a previous final set);
    the new elements n_prev..n-1 are clustered among themselves with
    Algorithm 2, and that set is merged into the previous one with one
    Algorithm 1 merge, the previous set first; then the final stage over the
    combined clusters.  Returns (clusters, similar pairs, stats of the new
    work)."""
    n = len(offsets) - 1
    judge = ProteinJudge(residues, offsets, M, T, mT, mU, go, ge)
    stats = Stats()
    # Algorithm 2 over the new elements alone: the FIFO schedule of n - n_prev
    # singletons, its set ids offset to the new elements
    sets = {k: [Cluster(n_prev + k, [n_prev + k])] for k in range(n - n_prev)}
    for first, second, result in merge_schedule(n - n_prev):
        sets[result] = merge(sets.pop(first), sets.pop(second), judge, stats)
    new_set = next(iter(sets.values())) if sets else []
    prev_set = [Cluster(int(r), [int(x) for x in m]) for r, m in prev]
    final = merge(prev_set, new_set, judge, stats) if new_set else prev_set
    pairs = similar_pairs(final, judge.score, T)
    return final, pairs, stats


def allvsall(residues, offsets, M, T=120, go=-11, ge=-1):
    """Ground truth: every (x, y), x < y, with score >= T."""
    from .sw import sw_batch
    n = len(offsets) - 1
    a, b = np.triu_indices(n, k=1)
    pr = np.stack([a, b], axis=1).astype(np.int32)
    sc = sw_batch(residues, offsets, pr, M, go, ge, with_end=False)
    keep = sc >= T
    return [(int(x), int(y), int(s)) for x, y, s in zip(a[keep], b[keep], sc[keep])]


def recall(found, truth):
    """|found intersect truth| / |truth| over (x, y) pairs (Section 6.1)."""
    f = {(x, y) for x, y, *_ in found}
    t = {(x, y) for x, y, *_ in truth}
    return len(f & t) / len(t) if t else 1.0


# ---------------------------------------------------------------------------
# screened variant: a pre-filter decides which candidate pairs are aligned
# ---------------------------------------------------------------------------
STAGE_REP, STAGE_EXCHANGE, STAGE_FINAL = 1, 2, 4


class ScreenedProteinJudge(ProteinJudge):
    """similar'(x, y) = (stage not screened or keep(x, y)) and score >= T."""

    def __init__(self, residues, offsets, M, keep, stages, T=120, mT=166, mU=15, go=-11, ge=-1,
                 min_product=0):
        super().__init__(residues, offsets, M, T, mT, mU, go, ge)
        self.keep = keep
        self.stages = stages
        self.min_product = min_product
        self._size = {}

    def begin_merge(self, cs1, cs2):
        # member counts at the start of the merge decide which representative
        # pairs bypass the screen
        self._size = {c.rep: len(c.objs) for c in list(cs1) + list(cs2)}

    def rep_test(self, r1, r2):
        guarded = self.min_product > 0 and self._size.get(r1, 1) * self._size.get(r2, 1) >= self.min_product
        if (self.stages & STAGE_REP) and not guarded and not self.keep(r1, r2):
            return (False, False, False)
        return super().rep_test(r1, r2)

    def member_similar(self, m, rep):
        if (self.stages & STAGE_EXCHANGE) and not self.keep(m, rep):
            return False
        return super().member_similar(m, rep)


def clustermerge_screened(residues, offsets, M, keep, stages, T=120, mT=166, mU=15, go=-11, ge=-1,
                          min_product=0):
    n = len(offsets) - 1
    judge = ScreenedProteinJudge(residues, offsets, M, keep, stages, T, mT, mU, go, ge, min_product)
    clusters, stats = bottom_up_merge(n, judge)
    out = []
    for x, y in cluster_pairs(clusters):
        if (stages & STAGE_FINAL) and not keep(x, y):
            continue
        s = judge.score(x, y)
        if s >= T:
            out.append((x, y, s))
    return clusters, out, stats
