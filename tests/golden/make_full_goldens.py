"""Write the expected outputs of the full-size parity tests.  Calls only the
oracle (``oracle/``) and the input recipes (``cmgen``); the Smith-Waterman
calls are spread over a process pool of independent oracle processes, which
changes nothing in the results (each score is one scalar oracle call).

  python tests/golden/make_full_goldens.py throughput   # 1,000,000 random pairs
  python tests/golden/make_full_goldens.py sets         # the family sets of SETS, or one by name
  python tests/golden/make_full_goldens.py cm20000      # 20,000-protein family set
  python tests/golden/make_full_goldens.py maxlen       # proteins of the longest accepted length

Outputs (next to this script):
  throughput_1m.json     SHA-256 of the scores and end cells of every pair row
                         (and of ten equal blocks of rows), cell count;
  <set name>.npz         clusters (final-set order), similar pairs and the
                         Algorithm 1 statistics of each family set of SETS
                         (2,000 proteins shaped like the 20,000-protein
                         workload, at several thresholds and a higher member
                         divergence; 400 proteins up to 5,000 residues);
  clustermerge_20000.json  digests of the clusters and similar pairs and the
                         statistics of the 20,000-protein set;
  max_length.json        score, end and start cells of every pair of the
                         longest-length set (cmgen.max_length_set).
Each file records the command, worker count and wall time.
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

import cmgen  # noqa: E402
import digest  # noqa: E402
from oracle import clustermerge as ocm  # noqa: E402
from oracle import sw_batch  # noqa: E402

_G = {}   # store of the forked workers


def _init(res, off, mat):
    _G["res"], _G["off"], _G["mat"] = res, off, mat


def _score_chunk(args):
    pairs, with_end = args
    return sw_batch(_G["res"], _G["off"], pairs, _G["mat"], with_end=with_end)


def _pool(ds, workers):
    ctx = mp.get_context("fork")
    _init(ds.residues, ds.offsets, ds.matrix)
    return ctx.Pool(workers)


def _chunks(pairs, size):
    return [pairs[k:k + size] for k in range(0, len(pairs), size)]


def throughput(workers: int):
    t0 = time.time()
    ds = cmgen.throughput_pool()
    L = ds.lengths()
    cells = float((L[ds.pairs[:, 0]] * L[ds.pairs[:, 1]]).sum())
    with _pool(ds, workers) as pool:
        parts = pool.map(_score_chunk, [(c, True) for c in _chunks(ds.pairs, 2000)], chunksize=1)
    sc = np.concatenate([p[0] for p in parts])
    ea = np.concatenate([p[1] for p in parts])
    eb = np.concatenate([p[2] for p in parts])
    out = dict(workload=ds.meta["workload"], seed=ds.meta["seed"], n_pairs=int(len(sc)), cells=cells,
               scores_sha256=digest.sha256_i32(sc), end_a_sha256=digest.sha256_i32(ea),
               end_b_sha256=digest.sha256_i32(eb), score_blocks=digest.block_hashes(sc),
               end_a_blocks=digest.block_hashes(ea), end_b_blocks=digest.block_hashes(eb),
               score_sum=int(sc.astype(np.int64).sum()), score_max=int(sc.max()),
               n_ge_120=int((sc >= 120).sum()), gap_open=-11, gap_extend=-1,
               command="python tests/golden/make_full_goldens.py throughput", workers=workers,
               wall_s=round(time.time() - t0, 1))
    with open(os.path.join(HERE, "throughput_1m.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("n_pairs", "cells", "wall_s", "score_max")}))


def _span_chunk(args):
    from oracle import span_batch
    return span_batch(_G["res"], _G["off"], args, _G["mat"])


def max_length(workers: int):
    t0 = time.time()
    ds = cmgen.max_length_set()
    with _pool(ds, workers) as pool:
        parts = pool.map(_span_chunk, [ds.pairs[k:k + 1] for k in range(len(ds.pairs))], chunksize=1)
    out5 = np.concatenate(parts)
    out = dict(workload=ds.meta["workload"], seed=ds.meta["seed"], lengths=ds.lengths().tolist(),
               pairs=ds.pairs.tolist(), score=out5[:, 0].tolist(), end_a=out5[:, 1].tolist(),
               end_b=out5[:, 2].tolist(), start_a=out5[:, 3].tolist(), start_b=out5[:, 4].tolist(),
               gap_open=-11, gap_extend=-1, command="python tests/golden/make_full_goldens.py maxlen",
               workers=workers, wall_s=round(time.time() - t0, 1))
    with open(os.path.join(HERE, "max_length.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("score", "wall_s")}))


class PoolJudge(ocm.ProteinJudge):
    """The oracle's protein judge with its score cache filled ahead of large
    merges: every representative pair of a merge's first set x second set
    (and, before the final stage, every in-cluster pair) is scored by the pool;
    the replay itself is the oracle's sequential Algorithms 1 and 2."""

    def __init__(self, ds, pool, min_batch=4096, **kw):
        super().__init__(ds.residues, ds.offsets, ds.matrix, **kw)
        self.pool = pool
        self.min_batch = min_batch
        self.prefetched = 0

    def fill(self, pairs):
        pairs = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
        if len(pairs) == 0:
            return
        size = max(256, min(20000, len(pairs) // (4 * self.pool._processes) + 1))
        parts = self.pool.map(_score_chunk, [(c, False) for c in _chunks(pairs, size)], chunksize=1)
        sc = np.concatenate(parts)
        for (x, y), s in zip(pairs.tolist(), sc.tolist()):
            self._score[(x, y) if x <= y else (y, x)] = s
        self.prefetched += len(pairs)

    def begin_merge(self, cs1, cs2):
        if len(cs1) * len(cs2) < self.min_batch:
            return
        r1 = np.array([c.rep for c in cs1], dtype=np.int64)
        r2 = np.array([c.rep for c in cs2], dtype=np.int64)
        a = np.repeat(r1, len(r2))
        b = np.tile(r2, len(r1))
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        key = np.unique(lo * (1 << 32) + hi)
        todo = [k for k in key.tolist() if (k >> 32, k & 0xffffffff) not in self._score]
        self.fill([(k >> 32, k & 0xffffffff) for k in todo])


def _cm_run(ds, workers, min_batch=4096, **kw):
    with _pool(ds, workers) as pool:
        judge = PoolJudge(ds, pool, min_batch=min_batch, **kw)
        t0 = time.time()
        clusters, stats = ocm.bottom_up_merge(ds.n, judge)
        t1 = time.time()
        print(f"merge tree done in {t1 - t0:.0f} s, {judge.prefetched} prefetched, {len(judge._score)} scores",
              flush=True)
        cand = ocm.cluster_pairs(clusters)
        todo = [p for p in cand if p not in judge._score]
        judge.fill(todo)
        pairs = ocm.similar_pairs(clusters, judge.score, judge.T)
        t2 = time.time()
        print(f"final stage done in {t2 - t1:.0f} s: {len(cand)} candidates, {len(pairs)} similar pairs", flush=True)
    return clusters, pairs, stats, len(cand), (t0, t1, t2)


def _stats_dict(stats, clusters, pairs, n_cand):
    return dict(rep_comparisons=stats.rep_comparisons, exchange_alignments=stats.exchange_alignments,
                full_merges=stats.full_merges, exchanges=stats.exchanges, n_clusters=len(clusters),
                final_candidates=n_cand, n_similar_pairs=len(pairs))


# family sets whose exact outputs are stored whole: name -> (generator kwargs, parameters)
SETS = {
    # the 20,000-protein workload's shape at 2,000 proteins
    "clustermerge_2000": (dict(n_seqs=2000, n_families=200, seed=212), dict(T=120, mT=166, mU=15)),
    # threshold sweep points (missed-pair sweep of Section 6.1)
    "clustermerge_2000_T100": (dict(n_seqs=2000, n_families=200, seed=212), dict(T=100, mT=140, mU=15)),
    "clustermerge_2000_T140": (dict(n_seqs=2000, n_families=200, seed=212), dict(T=140, mT=200, mU=15)),
    "clustermerge_2000_mU30": (dict(n_seqs=2000, n_families=200, seed=212), dict(T=120, mT=166, mU=30)),
    # more divergent families (dataset composition, Section 6.4)
    "clustermerge_2000_sub40": (dict(n_seqs=2000, n_families=200, seed=213, sub_rate=0.40),
                                dict(T=120, mT=166, mU=15)),
    # long proteins: lognormal median 1200, clipped to 30-5,000
    "clustermerge_long_400": (dict(n_seqs=400, n_families=40, seed=515, median=1200.0, hi=5000),
                              dict(T=120, mT=166, mU=15)),
}


def cm_set(name: str, workers: int):
    t0 = time.time()
    gen, par = SETS[name]
    ds = cmgen.clustermerge_families(**gen)
    clusters, pairs, stats, n_cand, _ = _cm_run(ds, workers, min_batch=64, **par)
    reps = np.array([c.rep for c in clusters], np.int32)
    moff = np.zeros(len(clusters) + 1, np.int64)
    np.cumsum([len(c.objs) for c in clusters], out=moff[1:])
    members = np.array([m for c in clusters for m in c.objs], np.int32)
    pa = np.array([(x, y, s) for x, y, s in pairs], np.int32).reshape(-1, 3)
    st = _stats_dict(stats, clusters, pairs, n_cand)
    info = dict(generator=gen, params=par, gap_open=-11, gap_extend=-1, max_len=int(ds.lengths().max()),
                command=f"python tests/golden/make_full_goldens.py {name}", workers=workers,
                wall_s=round(time.time() - t0, 1))
    np.savez_compressed(os.path.join(HERE, name + ".npz"), reps=reps, member_offsets=moff,
                        members=members, pairs=pa,
                        stats=np.array([st[k] for k in sorted(st)], np.int64),
                        stat_names=np.array(sorted(st)), info=np.array(json.dumps(info)))
    print(name, json.dumps(st), flush=True)


def cm20000(workers: int):
    t0 = time.time()
    ds = cmgen.clustermerge_families()
    clusters, pairs, stats, n_cand, (ta, tb, tc) = _cm_run(ds, workers)
    ca = digest.clusters_array([(c.rep, c.objs) for c in clusters])
    pa = np.array([(x, y, s) for x, y, s in pairs], np.int32).reshape(-1, 3)
    st = _stats_dict(stats, clusters, pairs, n_cand)
    out = dict(workload="clustermerge-20000: 2000 Zipf(1.2) families, lognormal median 350 sigma 0.6 clipped "
                        "30-2000", seed=202, T=120, mT=166, mU=15, gap_open=-11, gap_extend=-1,
               clusters_sha256=digest.sha256_i32(ca), pairs_sha256=digest.sha256_i32(digest.pairs_array(
                   pa[:, 0], pa[:, 1], pa[:, 2])),
               pair_blocks=digest.block_hashes(digest.pairs_array(pa[:, 0], pa[:, 1], pa[:, 2])),
               largest_cluster=int(max(len(c.objs) for c in clusters)), stats=st,
               command="python tests/golden/make_full_goldens.py cm20000", workers=workers,
               merge_s=round(tb - ta, 1), final_s=round(tc - tb, 1), wall_s=round(time.time() - t0, 1))
    with open(os.path.join(HERE, "clustermerge_20000.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(st))


if __name__ == "__main__":
    what = sys.argv[1]
    workers = int(sys.argv[2]) if len(sys.argv) > 2 else max(1, (os.cpu_count() or 2) - 1)
    if what in SETS:
        cm_set(what, workers)
    elif what == "sets":
        for name in SETS:
            cm_set(name, workers)
    else:
        {"throughput": throughput, "cm20000": cm20000, "maxlen": max_length}[what](workers)
