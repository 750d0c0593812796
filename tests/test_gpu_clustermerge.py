"""GPU ClusterMerge vs the sequential oracle (Algorithms 1 and 2, Section 6.1 final stage).

Exact equality of the final cluster list (representatives and member order),
of the similar-pair set with scores, and of the Algorithm 1 statistics.
"""
import numpy as np
import pytest

import cmgen
from oracle import clustermerge as ocm
from oracle import sw, sw_batch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1908_10574_amd as cm
    return cm


def dev_store(ds):
    res = torch.from_numpy(ds.residues.copy() if len(ds.residues) else np.zeros(1, np.uint8)).cuda()
    return res, torch.from_numpy(ds.offsets.copy()).cuda()


def run_both(cm, ds, T=120, mT=166, mU=15, ctx=None, rep_chunk_pairs=0):
    res, off = dev_store(ds)
    g = cm.clustermerge_run(res, off, ds.matrix, T=T, mT=mT, mU=mU, ctx=ctx, rep_chunk_pairs=rep_chunk_pairs)
    clusters, pairs, st = ocm.clustermerge(ds.residues, ds.offsets, ds.matrix, T=T, mT=mT, mU=mU)
    return g, clusters, pairs, st


def assert_same(g, clusters, pairs, st):
    got = [(r, list(m)) for r, m in g["clusters"]]
    want = [(c.rep, list(c.objs)) for c in clusters]
    assert len(got) == len(want)
    for k, (a, b) in enumerate(zip(got, want)):
        assert a == b, f"cluster {k}: gpu {a[0]} {a[1][:10]} oracle {b[0]} {b[1][:10]}"
    gp = [(int(x), int(y), int(s)) for (x, y), s in zip(g["pairs"], g["scores"])]
    assert gp == [tuple(p) for p in pairs]
    s = g["stats"]
    assert s["rep_comparisons"] == st.rep_comparisons
    assert s["exchange_alignments"] == st.exchange_alignments
    assert s["full_merges"] == st.full_merges
    assert s["exchanges"] == st.exchanges
    assert s["n_similar_pairs"] == len(pairs)
    assert s["n_clusters"] == len(clusters)


def test_small_families_exact(cm):
    ds = cmgen.allvsall_small()
    g, clusters, pairs, st = run_both(cm, ds)
    assert_same(g, clusters, pairs, st)
    truth, cells = cm.allvsall_count(*dev_store(ds), ds.matrix)
    otruth = ocm.allvsall(ds.residues, ds.offsets, ds.matrix)
    assert truth == len(otruth)
    L = ds.lengths().astype(np.float64)
    assert cells == pytest.approx((L.sum() ** 2 - (L ** 2).sum()) / 2)
    assert len(pairs) / truth > 0.9


@pytest.mark.parametrize("score_plan", [None, (1, 8), (0, 16)])
def test_zipf_families_exact(cm, score_plan):
    ds = cmgen.clustermerge_families(n_seqs=500, n_families=50, seed=212, median=120, hi=400)
    ctx = cm.Context(0)
    if score_plan:
        ctx.set_plan(0, score_plan[0], score_plan[1], 1)
        ctx.set_plan(0, score_plan[0], score_plan[1], ctx.get_plan(0)[3])
    g, clusters, pairs, st = run_both(cm, ds, ctx=ctx)
    assert_same(g, clusters, pairs, st)
    assert st.full_merges > 0 and st.exchanges > 0
    ctx.close()


@pytest.mark.parametrize("chunk", [-1, 1, 7, 300])
def test_chunked_representative_waves_exact(cm, chunk):
    """The representative pairs of a level aligned in column chunks (rows that
    left Algorithm 1's loop dropped from later chunks) give the oracle's result
    exactly; chunking only removes alignments that the replay never reads."""
    ds = cmgen.clustermerge_families(n_seqs=500, n_families=50, seed=212, median=120, hi=400)
    g, clusters, pairs, st = run_both(cm, ds, rep_chunk_pairs=chunk)
    assert_same(g, clusters, pairs, st)
    one = cm.clustermerge_run(*dev_store(ds), ds.matrix, rep_chunk_pairs=-1)
    assert g["stats"]["speculative_pairs"] <= one["stats"]["speculative_pairs"]
    if chunk in (1, 7):
        assert g["stats"]["aligned_pairs"] < one["stats"]["aligned_pairs"]
    for mT, mU in ((10**6, 15), (120, 400)):
        d2 = cmgen.clustermerge_families(n_seqs=160, n_families=20, seed=213, median=100, hi=300)
        g2, c2, p2, s2 = run_both(cm, d2, mT=mT, mU=mU, rep_chunk_pairs=chunk)
        assert_same(g2, c2, p2, s2)


@pytest.mark.parametrize("mT,mU", [(10**6, 15), (120, 400), (166, 0)])
def test_parameter_extremes_exact(cm, mT, mU):
    ds = cmgen.clustermerge_families(n_seqs=160, n_families=20, seed=213, median=100, hi=300)
    g, clusters, pairs, st = run_both(cm, ds, mT=mT, mU=mU)
    assert_same(g, clusters, pairs, st)
    if mT == 10**6:     # transitivity never holds: every pair meets once as representatives
        assert st.rep_comparisons == ds.n * (ds.n - 1) // 2
        truth, _ = cm.allvsall_count(*dev_store(ds), ds.matrix)
        assert len(pairs) == truth


def test_identical_proteins(cm):
    rng = np.random.default_rng(4)
    a = rng.integers(0, 20, size=60).astype(np.uint8)
    ds = cmgen.from_list([a] * 4)
    res, off = dev_store(ds)
    g = cm.clustermerge_run(res, off, ds.matrix)
    assert [(r, list(m)) for r, m in g["clusters"]] == [(3, [3, 2, 1, 0])]
    assert g["stats"]["rep_comparisons"] == 3
    assert len(g["pairs"]) == 6


@pytest.mark.parametrize("n_prev", [0, 1, 150, 400, 500])
def test_extend_exact(cm, n_prev):
    """New proteins classified against a previous clustering (Algorithm 2 over
    the new ones, one Algorithm 1 merge into the previous set, final stage):
    the GPU gives the oracle's clusters, pairs and statistics, and reuses the
    previous run's scores."""
    ds = cmgen.clustermerge_families(n_seqs=500, n_families=50, seed=212, median=120, hi=400)
    res, off = dev_store(ds)
    prev = cm.clustermerge_run(res, off[: n_prev + 1].contiguous(), ds.matrix) if n_prev else None
    pc = [(r, list(m)) for r, m in prev["clusters"]] if prev else []
    kw = dict(known_pairs=prev["pairs"], known_scores=prev["scores"]) if prev else {}
    g = cm.clustermerge_extend(res, off, ds.matrix, pc, n_prev, **kw)
    clusters, pairs, st = ocm.clustermerge_extend(ds.residues, ds.offsets, ds.matrix, pc, n_prev)
    assert_same(g, clusters, pairs, st)
    if 0 < n_prev < ds.n:
        assert g["stats"]["cache_hits"] >= len(prev["pairs"]) // 2
    if n_prev == 0:
        full = cm.clustermerge_run(res, off, ds.matrix)
        assert [(r, list(m)) for r, m in full["clusters"]] == [(r, list(m)) for r, m in g["clusters"]]


def test_extend_full_scale_properties(cm):
    """The 20,000-protein workload: its last 1,000 proteins classified against
    a clustering of the first 19,000.  Checks that hold at any size: a full
    merge moves whole clusters and an exchange copies members, so two members
    of a previous cluster always end in a common cluster and every previously
    found pair is found again, with the reused score; scores of pairs with a
    new protein equal the oracle's on a sample; the result repeats."""
    ds = cmgen.clustermerge_families()
    res, off = dev_store(ds)
    n_prev = 19000
    prev = cm.clustermerge_run(res, off[: n_prev + 1].contiguous(), ds.matrix)
    pc = [(r, list(m)) for r, m in prev["clusters"]]
    kw = dict(known_pairs=prev["pairs"], known_scores=prev["scores"])
    g = cm.clustermerge_extend(res, off, ds.matrix, pc, n_prev, **kw)
    s = g["stats"]
    pairs, scores = g["pairs"], g["scores"]
    assert (pairs[:, 0] < pairs[:, 1]).all() and (scores >= 120).all()
    key = pairs[:, 0].astype(np.int64) * ds.n + pairs[:, 1]
    assert (np.diff(key) > 0).all()
    pkey = prev["pairs"][:, 0].astype(np.int64) * ds.n + prev["pairs"][:, 1]
    at = np.searchsorted(key, pkey)
    assert (at < len(key)).all() and np.array_equal(key[at], pkey)
    assert np.array_equal(scores[at], prev["scores"])
    assert s["cache_hits"] >= len(pkey)
    seen = np.zeros(ds.n, bool)
    for r, m in g["clusters"]:
        ml = m.tolist()
        assert r in set(ml) and len(set(ml)) == len(ml)
        seen[m] = True
    assert seen.all()
    assert s["n_clusters"] <= len(pc) + (ds.n - n_prev)
    new = np.flatnonzero(pairs[:, 1] >= n_prev)
    assert len(new) > 0
    rng = np.random.default_rng(7)
    pick = new[rng.choice(len(new), size=min(300, len(new)), replace=False)]
    osc = sw_batch(ds.residues, ds.offsets, pairs[pick], ds.matrix, with_end=False)
    assert np.array_equal(osc, scores[pick])
    g2 = cm.clustermerge_extend(res, off, ds.matrix, pc, n_prev, **kw)
    assert g2["stats"]["pair_set_hash"] == s["pair_set_hash"]
    assert [(r, list(m)) for r, m in g2["clusters"]] == [(r, list(m)) for r, m in g["clusters"]]
    print({k: s[k] for k in ("n_clusters", "n_similar_pairs", "cache_hits", "final_candidates", "t_total_s")},
          len(prev["pairs"]), len(new))


def test_extend_rejects_inconsistent_clustering(cm):
    ds = cmgen.clustermerge_families(n_seqs=60, n_families=8, seed=215, median=100, hi=200)
    res, off = dev_store(ds)
    prev = cm.clustermerge_run(res, off[:41].contiguous(), ds.matrix)
    pc = [(r, list(m)) for r, m in prev["clusters"]]
    bad_cases = [
        pc[1:] if len(pc) > 1 else [],                                  # an element in no cluster
        [(pc[0][0], [x for x in pc[0][1] if x != pc[0][0]] or [45])] + pc[1:],   # rep not a member / out of range
        [(pc[0][0], pc[0][1] + [pc[0][1][0]])] + pc[1:],               # a member listed twice
    ]
    for bad in bad_cases:
        with pytest.raises(cm.CMError):
            cm.clustermerge_extend(res, off, ds.matrix, bad, 40)
    with pytest.raises(cm.CMError):
        cm.clustermerge_extend(res, off, ds.matrix, pc, 40, known_pairs=np.array([[0, 50]]), known_scores=[7])
    g = cm.clustermerge_extend(res, off, ds.matrix, pc, 40)           # the consistent one runs
    assert g["stats"]["n_clusters"] >= 1


def test_asymmetric_matrix_rejected(cm):
    """One score serves both orientations of a pair, so ClusterMerge refuses an
    asymmetric matrix before any work is enqueued."""
    ds = cmgen.family_dataset(3, [3] * 3, lambda r: 60, 30, 120, 71)
    res, off = dev_store(ds)
    M = ds.matrix.copy()
    M[2, 5] += 1
    with pytest.raises(cm.CMError, match="symmetric"):
        cm.clustermerge_run(res, off, M)
    g = cm.clustermerge_run(res, off, ds.matrix)     # the symmetric one runs
    assert g["stats"]["n_clusters"] >= 1


@pytest.mark.parametrize("n", [1, 2, 3])
def test_tiny_inputs(cm, n):
    ds = cmgen.clustermerge_families(n_seqs=n, n_families=1, seed=214, median=80, hi=200) if n > 0 else None
    g, clusters, pairs, st = run_both(cm, ds)
    assert_same(g, clusters, pairs, st)


def test_full_scale_20k_properties(cm):
    """The 20,000-protein workload: checks that hold at any size, oracle on a sample."""
    ds = cmgen.clustermerge_families()
    res, off = dev_store(ds)
    g = cm.clustermerge_run(res, off, ds.matrix)
    s = g["stats"]
    pairs, scores = g["pairs"], g["scores"]
    assert s["n_similar_pairs"] == len(pairs) > 0
    assert (pairs[:, 0] < pairs[:, 1]).all()
    key = pairs[:, 0].astype(np.int64) * ds.n + pairs[:, 1]
    assert (np.diff(key) > 0).all()          # sorted and unique
    assert (scores >= 120).all()
    rng = np.random.default_rng(5)
    pick = rng.choice(len(pairs), size=min(300, len(pairs)), replace=False)
    osc = sw_batch(ds.residues, ds.offsets, pairs[pick], ds.matrix, with_end=False)
    assert np.array_equal(osc, scores[pick])
    # every element is in some cluster; every member appears once per cluster
    seen = np.zeros(ds.n, bool)
    for r, m in g["clusters"]:
        assert r in set(m.tolist()) and len(set(m.tolist())) == len(m)
        seen[m] = True
    assert seen.all()
    assert s["rep_comparisons"] < ds.n * (ds.n - 1) // 2
    # deterministic: same result hash on a second run
    g2 = cm.clustermerge_run(res, off, ds.matrix)
    assert g2["stats"]["pair_set_hash"] == s["pair_set_hash"]
    assert g2["stats"]["rep_comparisons"] == s["rep_comparisons"]
    print({k: s[k] for k in ("rep_comparisons", "exchange_alignments", "full_merges", "exchanges", "rounds",
                             "waves", "aligned_pairs", "aligned_cells", "n_clusters", "n_similar_pairs",
                             "t_total_s", "t_gpu_s", "t_host_s")})


def _oracle_logit_table(ds, w):
    from oracle import screen as S
    f = S.features(ds.residues, ds.offsets)
    a, b = np.triu_indices(ds.n, k=1)
    pairs = np.stack([a, b], 1)
    z = np.concatenate([S.forward(w, S.pair_input(f, pairs[k:k + 4000]))[0] for k in range(0, len(pairs), 4000)])
    tab = np.full((ds.n, ds.n), np.nan)
    tab[a, b] = z
    tab[b, a] = z
    return tab, z


def ternary_weights(seed):
    """Weights in {-1, 0, 1}, zero biases: with features that are multiples of
    1/8, every input, hidden value and logit is a multiple of 1/64 small enough
    to be exact in fp32, so both sides compute identical logits."""
    from oracle import screen as S
    rng = np.random.default_rng(seed)
    w = rng.choice(np.array([-1.0, 0.0, 1.0], np.float32), size=S.n_params(), p=[0.2, 0.6, 0.2])
    p = S.unflatten(w)
    for b in ("b1", "b2", "b3"):
        p[b][...] = 0
    return S.flatten(p).astype(np.float32)


@pytest.mark.parametrize("stages,min_product,chunk", [(1, 0, 0), (2, 0, 0), (3, 0, 0), (7, 0, 0), (3, 4, 0), (1, 2, 0),
                                                     (3, 0, 5), (1, 4, 40)])
def test_screened_exact_vs_oracle_replay(cm, stages, min_product, chunk):
    """Same weights (drawn on the CPU) on both sides; keep decisions from each side's own MLP."""
    ds = cmgen.clustermerge_families(n_seqs=160, n_families=20, seed=213, median=100, hi=300)
    w = ternary_weights(21)
    tab, z = _oracle_logit_table(ds, w)
    assert np.array_equal(z * 64, np.round(z * 64))        # exact multiples of 1/64
    tau = float(np.median(z)) + 1.0 / 128
    scr = cm.Screen(0)
    scr.set_weights(w)
    res, off = dev_store(ds)
    a, b = np.triu_indices(ds.n, k=1)
    zg = scr.infer(cm.kmer_features(res, off), torch.from_numpy(np.stack([a, b], 1).astype(np.int32)).cuda())
    assert np.array_equal(zg.cpu().numpy(), z.astype(np.float32))
    g = cm.clustermerge_run(res, off, ds.matrix, screen=scr, screen_stages=stages, screen_tau=tau,
                            screen_min_product=min_product, rep_chunk_pairs=chunk)
    keep = lambda x, y: tab[x, y] >= tau  # noqa: E731
    clusters, pairs, st = ocm.clustermerge_screened(ds.residues, ds.offsets, ds.matrix, keep, stages,
                                                    min_product=min_product)
    assert_same(g, clusters, pairs, st)
    assert g["stats"]["screened_out"] > 0


def test_graph_replay_exact(cm):
    """Waves replayed as captured hipGraphs give the oracle's result, run after run."""
    ds = cmgen.clustermerge_families(n_seqs=500, n_families=50, seed=212, median=120, hi=400)
    ctx = cm.Context(0)
    ctx.set_graphs(True)
    res, off = dev_store(ds)
    clusters, pairs, st = ocm.clustermerge(ds.residues, ds.offsets, ds.matrix)
    for chunk in (0, 0, 3):
        g = cm.clustermerge_run(res, off, ds.matrix, ctx=ctx, rep_chunk_pairs=chunk)
        assert_same(g, clusters, pairs, st)
    ctx.close()


def test_graph_replay_matches_eager_20k(cm):
    ds = cmgen.clustermerge_families()
    res, off = dev_store(ds)
    eager = cm.clustermerge_run(res, off, ds.matrix)
    ctx = cm.Context(0)
    ctx.set_graphs(True)
    for _ in range(2):
        g = cm.clustermerge_run(res, off, ds.matrix, ctx=ctx)
        # captured waves send host-built pairs and align exchange requests in
        # their own waves; eager waves generate representative pairs on the
        # device (cells from per-merge length sums) and carry exchange requests
        for k in ("pair_set_hash", "n_similar_pairs", "rep_comparisons", "exchange_alignments", "full_merges",
                  "exchanges", "n_clusters", "aligned_pairs", "aligned_cells", "cache_hits", "end_pairs"):
            assert g["stats"][k] == eager["stats"][k], k
        assert all(r1 == r2 and np.array_equal(m1, m2) for (r1, m1), (r2, m2) in zip(g["clusters"], eager["clusters"]))
    print("graph", g["stats"]["t_total_s"], "eager", eager["stats"]["t_total_s"])
    ctx.close()


@pytest.mark.parametrize("graphs", [False, True])
def test_end_records_beyond_prefix(cm, graphs):
    """9,000 identical proteins: the first tree level has 4,500 merges whose single
    representative pair scores above mT, more end records than the copy that returns
    with the scores holds, so the rest is fetched separately.  Every merge is a full
    merge: one cluster, n - 1 comparisons, every pair similar."""
    n = 9000
    rng = np.random.default_rng(5)
    a = rng.integers(0, 20, size=30).astype(np.uint8)
    ds = cmgen.from_list([a] * n)
    assert int(ds.matrix[a, a].sum()) > 166
    res, off = dev_store(ds)
    ctx = cm.Context(0)
    ctx.set_graphs(graphs)
    g = cm.clustermerge_run(res, off, ds.matrix, max_result_pairs=0, ctx=ctx)
    judge = ocm.ProteinJudge(ds.residues, ds.offsets, ds.matrix)
    clusters, st = ocm.bottom_up_merge(n, judge)
    assert [(c.rep, c.objs) for c in clusters] == [(int(r), list(m)) for r, m in g["clusters"]]
    assert g["stats"]["rep_comparisons"] == st.rep_comparisons == n - 1
    assert g["stats"]["full_merges"] == n - 1
    assert g["stats"]["end_pairs"] == n - 1
    assert g["stats"]["n_similar_pairs"] == n * (n - 1) // 2
    ctx.close()


def test_allocation_failure_returns_enomem_and_context_recovers(cm, monkeypatch):
    """An allocation that fails inside cm_clustermerge_run (a host vector of the
    final stage while a batch is on the device, or the growth of device
    scratch) returns CM_ENOMEM instead of aborting; the same context then runs
    the same input to the exact result."""
    ds = cmgen.clustermerge_families(n_seqs=300, n_families=30, seed=231, median=120, hi=400)
    res, off = dev_store(ds)
    clusters, pairs, st = ocm.clustermerge(ds.residues, ds.offsets, ds.matrix)
    ctx = cm.Context(0)
    for site in ("device", "host"):   # device first: a fresh context still has scratch to grow
        monkeypatch.setenv("CM_TEST_FAIL_ALLOC", site)
        with pytest.raises(cm.CMError) as e:
            cm.clustermerge_run(res, off, ds.matrix, ctx=ctx)
        assert e.value.status == cm.CM_ENOMEM, (site, str(e.value))
        monkeypatch.delenv("CM_TEST_FAIL_ALLOC")
        g = cm.clustermerge_run(res, off, ds.matrix, ctx=ctx)
        assert_same(g, clusters, pairs, st)
    ctx.close()


def test_required_cells_closed_form(cm):
    """With T out of reach nothing is ever similar: Algorithm 2 compares every
    pair of proteins exactly once as representatives, there is no exchange and
    every final cluster is a singleton, so the cells the method needs are
    sum over x < y of L_x L_y; executed cells are at least that."""
    ds = cmgen.clustermerge_families(n_seqs=150, n_families=15, seed=241, median=150, hi=600)
    res, off = dev_store(ds)
    g = cm.clustermerge_run(res, off, ds.matrix, T=10 ** 6, mT=10 ** 6)
    s = g["stats"]
    L = ds.lengths().astype(np.float64)
    want = (L.sum() ** 2 - (L ** 2).sum()) / 2
    assert s["rep_comparisons"] == ds.n * (ds.n - 1) // 2 and s["exchanges"] == 0
    assert s["required_cells"] == want
    assert s["aligned_cells"] >= want
    # the workload's thresholds: required cells sit between the final stage's
    # share and the executed cells
    g = cm.clustermerge_run(res, off, ds.matrix)
    s = g["stats"]
    assert 0 < s["required_cells"] <= s["aligned_cells"]


def test_valu_probe_rates(cm):
    """The VALU probe's rates are positive and below what 256 compute units of
    128 lanes could issue at 3 GHz (packed 16-bit halves count twice; some
    32-bit adds issue above 64 lanes per clock on this chip)."""
    for kind, per_lane in ((cm.CM_PROBE_I32_ADD, 1), (cm.CM_PROBE_I32_MAX3, 1), (cm.CM_PROBE_PK16_ADD, 2),
                           (cm.CM_PROBE_PK16_MAX3, 2)):
        ops, clk = cm.probe_valu(kind)
        print(kind, ops / 1e12, "TOP/s", clk / 1e9, "GHz")
        assert 0 < ops < 256 * 128 * 3.0e9 * per_lane
        assert 0.5e9 < clk < 3.5e9


def test_recorded_candidates(cm):
    """record_candidates keeps every pair scored in the merge stage: a superset
    of the pairs the sequential oracle evaluates there (representative
    comparisons and exchange tests; the driver also scores speculative pairs),
    each with the oracle's score; the clustering itself is unchanged."""
    ds = cmgen.clustermerge_families(n_seqs=200, n_families=20, seed=243, median=120, hi=400)
    res, off = dev_store(ds)
    g = cm.clustermerge_run(res, off, ds.matrix, record_candidates=True)
    plain = cm.clustermerge_run(res, off, ds.matrix)
    assert g["stats"]["pair_set_hash"] == plain["stats"]["pair_set_hash"]
    assert "candidates" not in plain
    cand, sc = g["candidates"], g["candidate_scores"]
    assert (cand[:, 0] < cand[:, 1]).all()
    key = cand[:, 0].astype(np.int64) * ds.n + cand[:, 1]
    assert (np.diff(key) > 0).all()
    judge = ocm.ProteinJudge(ds.residues, ds.offsets, ds.matrix)
    ocm.bottom_up_merge(ds.n, judge)
    merge_pairs = set(judge._score)
    assert merge_pairs <= {(int(x), int(y)) for x, y in cand}
    assert np.array_equal(sc, sw_batch(ds.residues, ds.offsets, cand, ds.matrix, with_end=False))
