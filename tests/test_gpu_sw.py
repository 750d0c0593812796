"""GPU Smith-Waterman vs the CPU oracle: bit-exact scores, end cells and start cells.

All inputs are seeded synthetic proteins from cmgen; expected values come from
the scalar C oracle only.
"""
import numpy as np
import pytest

import cmgen
from oracle import sw_batch, span_batch

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1908_10574_amd as cm
    return cm


def to_dev(ds, pairs):
    res = torch.from_numpy(ds.residues.copy()).cuda() if len(ds.residues) else torch.zeros(1, dtype=torch.uint8).cuda()
    off = torch.from_numpy(ds.offsets.copy()).cuda()
    pr = torch.from_numpy(np.ascontiguousarray(pairs, dtype=np.int32)).cuda()
    return res, off, pr


def gpu_scores(cm, ds, pairs, go=-11, ge=-1, end=True, matrix=None):
    M = ds.matrix if matrix is None else matrix
    res, off, pr = to_dev(ds, pairs)
    out = cm.sw_score_batch(res, off, pr, M, go, ge, return_end=end)
    cm.sync()
    if end:
        return tuple(t.cpu().numpy() for t in out)
    return out.cpu().numpy()


def check_exact(cm, ds, pairs, go=-11, ge=-1, matrix=None, span=True, label=""):
    M = ds.matrix if matrix is None else matrix
    sc, ea, eb = gpu_scores(cm, ds, pairs, go, ge, True, M)
    osc, oea, oeb = sw_batch(ds.residues, ds.offsets, pairs, M, go, ge)
    bad = np.flatnonzero((sc != osc) | (ea != oea) | (eb != oeb))
    assert len(bad) == 0, f"{label}: {len(bad)} mismatches, first {pairs[bad[0]]} gpu {(sc[bad[0]], ea[bad[0]], eb[bad[0]])} oracle {(osc[bad[0]], oea[bad[0]], oeb[bad[0]])}"
    # score-only kernel agrees too
    s_only = gpu_scores(cm, ds, pairs, go, ge, False, M)
    assert np.array_equal(s_only, osc), label
    if span:
        res, off, pr = to_dev(ds, pairs)
        t_sc = torch.from_numpy(sc).cuda()
        t_ea = torch.from_numpy(ea).cuda()
        t_eb = torch.from_numpy(eb).cuda()
        sa, sb = cm.sw_span_batch(res, off, pr, M, t_sc, t_ea, t_eb, 0, go, ge)
        cm.sync()
        sa, sb = sa.cpu().numpy(), sb.cpu().numpy()
        ref = span_batch(ds.residues, ds.offsets, pairs, M, go, ge)
        bad = np.flatnonzero((sa != ref[:, 3]) | (sb != ref[:, 4]))
        assert len(bad) == 0, f"{label}: span mismatch at {pairs[bad[0]]}: gpu {(sa[bad[0]], sb[bad[0]])} oracle {tuple(ref[bad[0]])}"
    return sc


def test_allvsall_100_proteins(cm):
    ds = cmgen.allvsall_small()
    sc = check_exact(cm, ds, ds.pairs, label="allvsall-100")
    assert (sc >= cmgen.THRESHOLD).sum() > 100


def test_boundary_lengths(cm):
    """Lengths at every tile edge: lanes (16), strips (16*R rows, 256), chunks (16 columns)."""
    edges = [0, 1, 2, 3, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129, 191, 192, 193,
             255, 256, 257, 258, 300, 511, 512, 513, 767, 768, 769, 1023, 1025]
    rng = np.random.default_rng(31)
    anc = rng.integers(0, 20, size=1100).astype(np.uint8)
    seqs = []
    for L in edges:
        seqs.append(cmgen.mutate(rng, anc)[:L] if L else np.zeros(0, np.uint8))
        seqs.append(rng.integers(0, 20, size=L).astype(np.uint8))
    ds = cmgen.from_list(seqs)
    n = ds.n
    a, b = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pairs = np.stack([a.ravel(), b.ravel()], 1).astype(np.int32)
    keep = rng.random(len(pairs)) < 0.45
    check_exact(cm, ds, pairs[keep], label="edges")


@pytest.mark.parametrize("seed", [41, 42])
def test_fuzz_mixed_lengths(cm, seed):
    rng = np.random.default_rng(seed)
    fam = cmgen.family_dataset(12, [6] * 12, lambda r: int(r.integers(20, 900)), 1, 1200, seed)
    pool = cmgen.uniform_pool(40, 0, 700, seed + 100)
    seqs = [fam.seq(i) for i in range(fam.n)] + [pool.seq(i) for i in range(pool.n)]
    ds = cmgen.from_list(seqs)
    pairs = cmgen.random_pairs(rng, ds.n, 1500)
    check_exact(cm, ds, pairs, label=f"fuzz{seed}")


def test_ties_and_zero_scores(cm):
    """Residues whose mutual score is 0 and repeated motifs make many equal optima."""
    M = cmgen.make_matrix().copy()
    M[0, 1] = M[1, 0] = 0
    M[2, 3] = M[3, 2] = 0
    rng = np.random.default_rng(51)
    seqs = [rng.integers(0, 4, size=int(rng.integers(0, 300))).astype(np.uint8) for _ in range(50)]
    motif = rng.integers(0, 20, size=12).astype(np.uint8)
    seqs += [np.tile(motif, k) for k in range(1, 8)]
    ds = cmgen.from_list(seqs, M)
    pairs = cmgen.random_pairs(rng, ds.n, 1200)
    check_exact(cm, ds, pairs, label="ties")
    all_neg = -np.ones((20, 20), np.int32)
    sc = gpu_scores(cm, ds, pairs[:50], matrix=all_neg)
    assert (sc[0] == 0).all() and (sc[1] == -1).all()


@pytest.mark.parametrize("go,ge", [(-11, -1), (-5, -5), (-3, 0), (-1000000, -1), (-20, -2)])
def test_extreme_gap_parameters(cm, go, ge):
    ds = cmgen.family_dataset(6, [5] * 6, lambda r: int(r.integers(30, 400)), 1, 600, 61)
    rng = np.random.default_rng(62)
    pairs = cmgen.random_pairs(rng, ds.n, 400)
    check_exact(cm, ds, pairs, go, ge, label=f"gaps{go},{ge}")


def test_large_magnitude_matrix(cm):
    rng = np.random.default_rng(71)
    M = rng.integers(-127, 128, size=(20, 20)).astype(np.int32)
    ds = cmgen.uniform_pool(30, 1, 500, 72)
    pairs = cmgen.random_pairs(rng, ds.n, 300)
    check_exact(cm, ds, pairs, -30, -3, matrix=M, label="asymmetric +-127 matrix")


def test_long_multistrip_pairs(cm):
    """Queries spanning several 256-row strips, up to 5,000 residues."""
    rng = np.random.default_rng(81)
    anc = rng.integers(0, 20, size=5000).astype(np.uint8)
    seqs = [cmgen.mutate(rng, anc)[:L] for L in (700, 1500, 2600, 4000, 5000)]
    seqs += [rng.integers(0, 20, size=L).astype(np.uint8) for L in (1000, 3000, 5000)]
    ds = cmgen.from_list(seqs)
    a, b = np.meshgrid(np.arange(ds.n), np.arange(ds.n), indexing="ij")
    pairs = np.stack([a.ravel(), b.ravel()], 1).astype(np.int32)
    check_exact(cm, ds, pairs, label="long")


def test_maximum_length(cm):
    """Sequences at the longest accepted length (CM_MAX_LEN = 65,535; 128 strips
    of 512 rows in the shared-query kernel, 512 of 128 in the two-profile packed
    kernel, 256 of 256 in the int32 kernels): one query against eight subjects
    of 0.9-1.0 CM_MAX_LEN residues (one item of the shared-query kernel: an
    identical copy, whose score saturates 16 bits and is re-run in int32,
    mutated relatives and unrelated proteins), a stretch of the query, short
    partners both ways.  Expected values: the oracle's (stored by
    tests/golden/make_full_goldens.py maxlen) and the closed forms of a
    self-alignment and of an embedded stretch.  Every score plan, and the
    score+end and start-cell passes.  One residue more is rejected."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "max_length.json")))
    ds = cmgen.max_length_set()
    L = cm.CM_MAX_LEN
    assert ds.lengths().max() == L and ds.lengths().tolist() == gold["lengths"]
    assert ds.pairs.tolist() == gold["pairs"]
    want = np.array([gold[k] for k in ("score", "end_a", "end_b", "start_a", "start_b")]).T
    # closed forms: the query against its copy scores the sum of its diagonal
    # entries over the whole length; its stretch 20000..23999 scores its own
    # diagonal sum, ending on the stretch's last cell inside the query
    q = ds.seq(0)
    diag = int(ds.matrix[q, q].sum())
    k_self = gold["pairs"].index([0, 1])
    assert tuple(want[k_self]) == (diag, L - 1, L - 1, 0, 0)
    t = ds.seq(9)
    k_sub = gold["pairs"].index([9, 0])
    assert tuple(want[k_sub]) == (int(ds.matrix[t, t].sum()), len(t) - 1, 20000 + len(t) - 1, 0, 20000)
    res, off, pr = to_dev(ds, ds.pairs)
    for plan in ("default", (1, 8), (0, 16)):
        ctx = cm.Context(0)
        if plan != "default":
            ctx.set_plan(0, plan[0], plan[1], 1)
            ctx.set_plan(0, plan[0], plan[1], ctx.get_plan(0)[3])     # at its occupancy limit
        print("max length, score plan", plan, flush=True)
        sc = cm.sw_score_batch(res, off, pr, ds.matrix, ctx=ctx)
        ctx.sync()
        assert np.array_equal(sc.cpu().numpy(), want[:, 0]), plan
        ctx.close()
    print("max length, score+end and start cells", flush=True)
    sc, ea, eb = cm.sw_score_batch(res, off, pr, ds.matrix, return_end=True)
    sa, sb = cm.sw_span_batch(res, off, pr, ds.matrix, sc, ea, eb, 0)
    cm.sync()
    got = np.stack([x.cpu().numpy() for x in (sc, ea, eb, sa, sb)], 1)
    bad = np.flatnonzero((got != want).any(axis=1))
    assert len(bad) == 0, (ds.pairs[bad], got[bad], want[bad])
    assert want[:, 0].max() > 32767              # a saturated pair re-run in int32
    too_long = cmgen.from_list([np.zeros(L + 1, np.uint8), np.zeros(5, np.uint8)])
    res, off, pr = to_dev(too_long, np.array([[0, 1]], np.int32))
    cm.sw_score_batch(res, off, pr, too_long.matrix)
    with pytest.raises(cm.CMError) as e:
        cm.sync()
    assert e.value.status == cm.CM_ERANGE


def test_throughput_workload_sampled(cm):
    """Shapes of the 1M-pair throughput workload: a 4,000-pair slice, every pair checked."""
    ds = cmgen.throughput_pool(n_pool=4000, n_pairs=4000, seed=303)
    sc = check_exact(cm, ds, ds.pairs, span=False, label="throughput-slice")
    assert sc.max() < cmgen.THRESHOLD   # unrelated random proteins


def test_deterministic_repeat(cm):
    ds = cmgen.allvsall_small()
    a = gpu_scores(cm, ds, ds.pairs)
    b = gpu_scores(cm, ds, ds.pairs)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_empty_batch_and_empty_sequences(cm):
    ds = cmgen.from_list([np.zeros(0, np.uint8), np.arange(10, dtype=np.uint8)])
    res, off, pr = to_dev(ds, np.zeros((0, 2), np.int32))
    out = cm.sw_score_batch(res, off, pr, ds.matrix)
    cm.sync()
    assert out.numel() == 0
    sc, ea, eb = gpu_scores(cm, ds, np.array([[0, 1], [1, 0], [0, 0], [1, 1]], np.int32))
    assert list(sc[:3]) == [0, 0, 0] and list(ea[:3]) == [-1, -1, -1]
    assert sc[3] == int(ds.matrix[np.arange(10), np.arange(10)].sum())


def test_error_paths(cm):
    ds = cmgen.uniform_pool(4, 5, 10, 91)
    res, off, pr = to_dev(ds, np.array([[0, 1]], np.int32))
    with pytest.raises(cm.CMError) as e:
        cm.sw_score_batch(res, off, pr, ds.matrix, -11, 2)
    assert e.value.status == cm.CM_EINVAL
    with pytest.raises(cm.CMError) as e:
        cm.sw_score_batch(res, off, pr, ds.matrix, -1, -3)       # open cheaper than extend
    assert e.value.status == cm.CM_EINVAL
    big = ds.matrix.copy()
    big[0, 0] = 500
    with pytest.raises(cm.CMError) as e:
        cm.sw_score_batch(res, off, pr, big)
    assert e.value.status == cm.CM_EUNSUPPORTED
    # device-detected errors: index out of range, residue code >= 20
    _, _, bad_pairs = to_dev(ds, np.array([[0, 7], [1, 2]], np.int32))
    out = cm.sw_score_batch(res, off, bad_pairs, ds.matrix)
    with pytest.raises(cm.CMError) as e:
        cm.sync()
    assert e.value.status == cm.CM_ERANGE
    bad_res = res.clone()
    bad_res[int(ds.offsets[1])] = 25
    out = cm.sw_score_batch(bad_res, off, pr, ds.matrix)
    with pytest.raises(cm.CMError) as e:
        cm.sync()
    assert e.value.status == cm.CM_ERANGE
    cm.sync()   # flag was cleared
    out = cm.sw_score_batch(res, off, pr, ds.matrix)
    cm.sync()
    assert out.cpu().numpy()[0] == sw_batch(ds.residues, ds.offsets, np.array([[0, 1]], np.int32), ds.matrix, with_end=False)[0]


def test_throughput_full_size_sampled(cm):
    """The full 1,000,000-pair batch as timed by the benchmark: a seeded sample of
    outputs checked one by one against the oracle, and run-to-run identity."""
    ds = cmgen.throughput_pool()
    res, off, pr = to_dev(ds, ds.pairs)
    a = cm.sw_score_batch(res, off, pr, ds.matrix)
    b = cm.sw_score_batch(res, off, pr, ds.matrix)
    sc, ea, eb = cm.sw_score_batch(res, off, pr, ds.matrix, return_end=True)
    cm.sync()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(a, b) and np.array_equal(a, sc.cpu().numpy())
    rng = np.random.default_rng(7)
    L = ds.lengths()
    cost = L[ds.pairs[:, 0]].astype(np.float64) * L[ds.pairs[:, 1]]
    pick = np.concatenate([rng.choice(len(a), 300, replace=False), np.argsort(cost)[-20:], np.argsort(cost)[:20]])
    osc, oea, oeb = sw_batch(ds.residues, ds.offsets, ds.pairs[pick], ds.matrix)
    assert np.array_equal(a[pick], osc)
    assert np.array_equal(ea.cpu().numpy()[pick], oea) and np.array_equal(eb.cpu().numpy()[pick], oeb)


def test_packed_saturation_boundary(cm):
    """Scores around the limits of the packed score kernel.  With a +127
    diagonal, an identical pair of length L scores 127 L.  Packed values carry
    a bias of 128 and are exact below 0x7C00 = 31744, i.e. for scores below
    31616: 248 residues give 31496 (packed result), 249 give 31623 (recomputed
    by the int32 kernel), 258 give 32766 (recomputed), 259 give 32893 (the
    packed sums saturate; recomputed).  Saturating and ordinary pairs share
    groups."""
    M = np.full((20, 20), -7, np.int32)
    np.fill_diagonal(M, 127)
    rng = np.random.default_rng(97)
    lens = [247, 248, 249, 250, 257, 258, 259, 260, 300, 1000, 4000]
    seqs = []
    for L in lens:
        s = rng.integers(0, 20, size=L).astype(np.uint8)
        seqs += [s, s.copy(), rng.integers(0, 20, size=L).astype(np.uint8)]
    ds = cmgen.from_list(seqs, M)
    pairs = []
    for k in range(len(lens)):
        a, b, c = 3 * k, 3 * k + 1, 3 * k + 2
        pairs += [(a, b), (b, a), (a, a), (a, c), (c, b), (c, c)]
    pairs = np.array(pairs * 3, np.int32)
    res, off, pr = to_dev(ds, pairs)
    sc = cm.sw_score_batch(res, off, pr, M)
    cm.sync()
    ref = sw_batch(ds.residues, ds.offsets, pairs, M, with_end=False)
    assert np.array_equal(sc.cpu().numpy(), ref)
    assert (ref > 32767).sum() > 10 and ((ref >= 31616) & (ref < 32767)).sum() >= 6
    assert ((ref > 31000) & (ref < 31616)).sum() >= 6
    ctx = cm.context()
    saved = ctx.get_plan(0)
    try:
        for kind, rmax in ((1, 4), (1, 8), (2, 32)):
            ctx.set_plan(0, kind, rmax, 1)
            sc = cm.sw_score_batch(res, off, pr, M)
            cm.sync()
            assert np.array_equal(sc.cpu().numpy(), ref), (kind, rmax)
    finally:
        ctx.set_plan(0, saved[0], saved[1], saved[2])


def test_cells_computed_accounting(cm):
    """The kernels' count of computed cells follows the strip and skew layout.
    Eight copies of one 100 x 100 pair: on the two-profile packed kernel (at
    most 8 rows per lane) they are one item of one strip of 7 rows per lane
    and 116 column steps (100 + 15, rounded up to even) over 64 lanes and two
    halves; their score+end pass has 8 pairs, at most four per wavefront, so
    each pair takes a whole 64-lane wavefront with 2 rows per lane and 164
    steps (100 + 63, rounded up to even).  Both are above the 80,000 cells the
    pairs have, and the scores stay the oracle's."""
    rng = np.random.default_rng(7)
    ds = cmgen.from_list([rng.integers(0, 20, size=100).astype(np.uint8),
                          rng.integers(0, 20, size=100).astype(np.uint8)])
    pairs = np.array([(0, 1)] * 8, np.int32)
    res, off, pr = to_dev(ds, pairs)
    ctx = cm.Context(0)
    ctx.set_plan(0, 1, 8, 1)
    c0 = ctx.cells_computed(0)
    sc = cm.sw_score_batch(res, off, pr, ds.matrix, ctx=ctx)
    ctx.sync()
    assert ctx.cells_computed(0) - c0 == 116 * 128 * 7
    c1 = ctx.cells_computed(1)
    s2, ea, eb = cm.sw_score_batch(res, off, pr, ds.matrix, return_end=True, ctx=ctx)
    ctx.sync()
    assert ctx.cells_computed(1) - c1 == 8 * 164 * 64 * 2
    osc, oea, oeb = sw_batch(ds.residues, ds.offsets, pairs, ds.matrix, -11, -1)
    assert np.array_equal(sc.cpu().numpy(), osc) and np.array_equal(s2.cpu().numpy(), osc)
    assert np.array_equal(ea.cpu().numpy(), oea) and np.array_equal(eb.cpu().numpy(), oeb)
    ctx.close()
