"""Exact parity at full size against stored oracle outputs.

The expected values were written by ``tests/golden/make_full_goldens.py``,
which runs only the CPU oracle (Smith-Waterman calls spread over a process
pool).  Nothing here is sampled:
  * every score and end cell of the 1,000,000-pair throughput batch (score-only
    launch as the benchmark times it, and the score+end launch);
  * the whole output (clusters in final-set order, similar pairs with scores,
    Algorithm 1 statistics) of 2,000-protein family sets shaped like the
    20,000-protein workload, at the workload's thresholds, at the missed-pair
    sweep's T = 100 and T = 140, at mU = 30, with more divergent families, and
    of 400 proteins up to 5,000 residues long;
  * digests of the clusters and similar pairs, and the statistics, of the
    full 20,000-protein workload.
"""
import json
import os
import sys

import numpy as np
import pytest

import cmgen

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")
sys.path.insert(0, GOLD)
import digest  # noqa: E402
from make_full_goldens import SETS  # noqa: E402

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1908_10574_amd as cm
    return cm


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _first_bad_block(got, want_blocks):
    have = digest.block_hashes(got, len(want_blocks))
    return [k for k, (a, b) in enumerate(zip(have, want_blocks)) if a != b]


def test_throughput_1m_every_output(cm):
    path = os.path.join(GOLD, "throughput_1m.json")
    gold = json.load(open(path))
    ds = cmgen.throughput_pool()
    assert len(ds.pairs) == gold["n_pairs"]
    res, off, pr = dev(ds.residues), dev(ds.offsets), dev(ds.pairs)
    print("throughput: score-only launch", flush=True)
    sc = cm.sw_score_batch(res, off, pr, ds.matrix)
    cm.sync()
    sc = sc.cpu().numpy()
    assert digest.sha256_i32(sc) == gold["scores_sha256"], _first_bad_block(sc, gold["score_blocks"])
    print("throughput: score+end launch", flush=True)
    s2, ea, eb = cm.sw_score_batch(res, off, pr, ds.matrix, return_end=True)
    cm.sync()
    s2, ea, eb = s2.cpu().numpy(), ea.cpu().numpy(), eb.cpu().numpy()
    assert digest.sha256_i32(s2) == gold["scores_sha256"], _first_bad_block(s2, gold["score_blocks"])
    assert digest.sha256_i32(ea) == gold["end_a_sha256"], _first_bad_block(ea, gold["end_a_blocks"])
    assert digest.sha256_i32(eb) == gold["end_b_sha256"], _first_bad_block(eb, gold["end_b_blocks"])


def _load_set(name):
    z = np.load(os.path.join(GOLD, name + ".npz"), allow_pickle=False)
    stats = dict(zip([str(s) for s in z["stat_names"]], z["stats"].tolist()))
    clusters = [(int(z["reps"][k]), z["members"][z["member_offsets"][k]:z["member_offsets"][k + 1]].tolist())
                for k in range(len(z["reps"]))]
    return clusters, z["pairs"], stats, json.loads(str(z["info"]))


def _assert_result(g, clusters, pairs, stats):
    got = [(int(r), [int(x) for x in m]) for r, m in g["clusters"]]
    assert len(got) == len(clusters)
    for k, (a, b) in enumerate(zip(got, clusters)):
        assert a == b, f"cluster {k}: gpu {a[0]} {a[1][:10]} oracle {b[0]} {b[1][:10]}"
    gp = np.concatenate([np.asarray(g["pairs"], np.int32).reshape(-1, 2),
                         np.asarray(g["scores"], np.int32).reshape(-1, 1)], axis=1)
    assert gp.shape == pairs.shape and np.array_equal(gp, pairs)
    s = g["stats"]
    for k in ("rep_comparisons", "exchange_alignments", "full_merges", "exchanges", "n_clusters",
              "final_candidates", "n_similar_pairs"):
        assert s[k] == stats[k], (k, s[k], stats[k])


@pytest.mark.parametrize("name", sorted(SETS))
def test_family_sets_exact(cm, name):
    clusters, pairs, stats, info = _load_set(name)
    gen, par = SETS[name]
    assert info["generator"] == json.loads(json.dumps(gen)) and info["params"] == par
    ds = cmgen.clustermerge_families(**gen)
    res, off = dev(ds.residues), dev(ds.offsets)
    print(name, par, flush=True)
    g = cm.clustermerge_run(res, off, ds.matrix, **par)
    _assert_result(g, clusters, pairs, stats)


def test_family_set_2000_under_other_launch_choices(cm):
    """The same exact output with graph-captured waves, with representative
    waves cut into small column chunks (eager: pairs built on the device;
    captured: on the host, which must align the same pairs and cells), and
    with the two-profile packed and the int32 score kernels."""
    clusters, pairs, stats, _ = _load_set("clustermerge_2000")
    gen, par = SETS["clustermerge_2000"]
    ds = cmgen.clustermerge_families(**gen)
    res, off = dev(ds.residues), dev(ds.offsets)
    chunk_stats = {}
    for variant in ("graphs", "chunks", "graphs_chunks", "packed1", "int32"):
        print(variant, flush=True)
        ctx = cm.Context(0)
        kw = {}
        if variant == "graphs":
            ctx.set_graphs(True)
        elif variant in ("chunks", "graphs_chunks"):
            kw["rep_chunk_pairs"] = 5000
            ctx.set_graphs(variant == "graphs_chunks")
        elif variant == "packed1":
            ctx.set_plan(0, 1, 8, 1)
            ctx.set_plan(0, 1, 8, ctx.get_plan(0)[3])
        else:
            ctx.set_plan(0, 0, 16, 1)
            ctx.set_plan(0, 0, 16, ctx.get_plan(0)[3])
        g = cm.clustermerge_run(res, off, ds.matrix, ctx=ctx, **par, **kw)
        _assert_result(g, clusters, pairs, stats)
        if "chunks" in variant:
            chunk_stats[variant] = (g["stats"]["aligned_pairs"], g["stats"]["aligned_cells"])
        ctx.close()
    assert chunk_stats["chunks"] == chunk_stats["graphs_chunks"], chunk_stats


def test_clustermerge_20000_digest(cm):
    path = os.path.join(GOLD, "clustermerge_20000.json")
    if not os.path.exists(path):
        pytest.skip("clustermerge_20000.json not written yet (make_full_goldens.py cm20000, about an hour)")
    gold = json.load(open(path))
    ds = cmgen.clustermerge_families()
    res, off = dev(ds.residues), dev(ds.offsets)
    print("clustermerge 20000", flush=True)
    g = cm.clustermerge_run(res, off, ds.matrix, T=gold["T"], mT=gold["mT"], mU=gold["mU"])
    s = g["stats"]
    for k, v in gold["stats"].items():
        assert s[k] == v, (k, s[k], v)
    ca = digest.clusters_array(g["clusters"])
    assert digest.sha256_i32(ca) == gold["clusters_sha256"]
    pa = digest.pairs_array(g["pairs"][:, 0], g["pairs"][:, 1], g["scores"])
    assert digest.sha256_i32(pa) == gold["pairs_sha256"], _first_bad_block(pa, gold["pair_blocks"])
