"""GPU alignment columns (cm_sw_traceback_batch) vs the CPU oracle's traceback:
identical column strings for every pair, ties included."""
import numpy as np
import pytest

import cmgen
from oracle import traceback_batch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1908_10574_amd as cm
    return cm


def gpu_columns(cm, ds, pairs, M=None, go=-11, ge=-1):
    M = ds.matrix if M is None else M
    res = torch.from_numpy(ds.residues.copy()).cuda()
    off = torch.from_numpy(ds.offsets.copy()).cuda()
    pr = torch.from_numpy(np.ascontiguousarray(pairs, dtype=np.int32)).cuda()
    sc, ea, eb = cm.sw_score_batch(res, off, pr, M, go, ge, return_end=True)
    sa, sb = cm.sw_span_batch(res, off, pr, M, sc, ea, eb, 0, go, ge)
    ops, op_off, n_ops = cm.sw_traceback_batch(res, off, pr, M, sc, ea, eb, sa, sb, go, ge)
    cm.sync()
    return cm.columns_as_strings(ops, op_off, n_ops), n_ops.cpu().numpy()


def check(cm, ds, pairs, M=None, go=-11, ge=-1, label=""):
    M = ds.matrix if M is None else M
    got, n_ops = gpu_columns(cm, ds, pairs, M, go, ge)
    want, span = traceback_batch(ds.residues, ds.offsets, pairs, M, go, ge)
    bad = [k for k in range(len(pairs)) if got[k] != want[k]]
    assert not bad, f"{label}: {len(bad)} mismatches, first {pairs[bad[0]]}: gpu {got[bad[0]][:60]} oracle {want[bad[0]][:60]}"
    assert (n_ops >= 0).all()
    return got


def test_allvsall_100(cm):
    ds = cmgen.allvsall_small()
    got = check(cm, ds, ds.pairs, label="allvsall-100")
    assert sum(1 for g in got if "I" in g or "D" in g) > 100


@pytest.mark.parametrize("go,ge", [(-11, -1), (-5, -5), (-3, 0), (-1, -1)])
def test_mixed_lengths_and_gap_models(cm, go, ge):
    rng = np.random.default_rng(601)
    fam = cmgen.family_dataset(10, [5] * 10, lambda r: int(r.integers(20, 700)), 1, 900, 602)
    pool = cmgen.uniform_pool(20, 0, 500, 603)
    ds = cmgen.from_list([fam.seq(i) for i in range(fam.n)] + [pool.seq(i) for i in range(pool.n)])
    pairs = cmgen.random_pairs(rng, ds.n, 800)
    check(cm, ds, pairs, go=go, ge=ge, label=f"mixed {go},{ge}")


def test_ties(cm):
    """Repeats around cheap gaps: many equally good alignments; the GPU walk
    picks the oracle's."""
    M = cmgen.make_matrix().copy()
    M[0, 1] = M[1, 0] = 0
    M[2, 3] = M[3, 2] = 0
    rng = np.random.default_rng(604)
    motif = rng.integers(0, 20, size=7).astype(np.uint8)
    seqs = [rng.integers(0, 4, size=int(rng.integers(1, 60))).astype(np.uint8) for _ in range(40)]
    seqs += [np.concatenate([np.tile(motif, k), rng.integers(0, 20, size=3).astype(np.uint8), np.tile(motif, 3)])
             for k in range(1, 6)]
    ds = cmgen.from_list(seqs, M)
    pairs = cmgen.random_pairs(rng, ds.n, 1500)
    for go, ge in ((-2, -1), (-1, -1), (-11, -1)):
        check(cm, ds, pairs, M, go, ge, label=f"ties {go},{ge}")


def test_long_pairs(cm):
    rng = np.random.default_rng(605)
    anc = rng.integers(0, 20, size=4000).astype(np.uint8)
    seqs = [cmgen.mutate(rng, anc)[:L] for L in (1500, 2600, 4000)] + [rng.integers(0, 20, size=3000).astype(np.uint8)]
    ds = cmgen.from_list(seqs)
    pairs = np.array([(0, 1), (1, 2), (2, 0), (3, 0), (2, 2)], np.int32)
    got = check(cm, ds, pairs, label="long")
    assert got[4] == "M" * 4000


def test_found_pairs_of_clustermerge(cm):
    """Pairs reported by a ClusterMerge run (similar pairs within clusters)."""
    ds = cmgen.clustermerge_families(n_seqs=500, n_families=50, seed=212, median=120, hi=400)
    res = torch.from_numpy(ds.residues).cuda()
    off = torch.from_numpy(ds.offsets).cuda()
    g = cm.clustermerge_run(res, off, ds.matrix)
    pairs = g["pairs"]
    rng = np.random.default_rng(606)
    pick = pairs[rng.choice(len(pairs), size=min(3000, len(pairs)), replace=False)]
    check(cm, ds, pick, label="clustermerge pairs")


def test_full_scale_found_pairs(cm):
    """The 20,000-protein ClusterMerge workload: 200,000 of its found pairs
    sampled as the benchmark's traceback leg does (one call) plus the 500
    largest boxes.  Every pair: its columns are an alignment of its box that
    scores exactly its Smith-Waterman score (the batch checker); a sample:
    the oracle's columns, spans and scores."""
    from alignment_columns import check_columns
    ds = cmgen.clustermerge_families()
    res = torch.from_numpy(ds.residues).cuda()
    off = torch.from_numpy(ds.offsets).cuda()
    g = cm.clustermerge_run(res, off, ds.matrix)
    found, fscore = g["pairs"], g["scores"]
    rng = np.random.default_rng(11)
    lens = np.diff(ds.offsets)
    idx = np.concatenate([rng.choice(len(found), size=min(200000, len(found)), replace=False),
                          np.argsort(lens[found[:, 0]] * lens[found[:, 1]], kind="stable")[-500:]])
    pick = np.ascontiguousarray(found[idx], dtype=np.int32)
    print(f"full-scale traceback: {len(pick)} pairs", flush=True)
    pr = torch.from_numpy(pick).cuda()
    sc, ea, eb = cm.sw_score_batch(res, off, pr, ds.matrix, return_end=True)
    sa, sb = cm.sw_span_batch(res, off, pr, ds.matrix, sc, ea, eb, 0)
    ops, op_off, n_ops = cm.sw_traceback_batch(res, off, pr, ds.matrix, sc, ea, eb, sa, sb)
    cm.sync()
    span = torch.stack([sc, ea, eb, sa, sb], 1).cpu().numpy()
    assert np.array_equal(span[:, 0], fscore[idx])     # the scores ClusterMerge recorded
    ops_h, off_h, n_h = ops.cpu().numpy(), op_off.cpu().numpy(), n_ops.cpu().numpy()
    step = 25000
    for k in range(0, len(pick), step):
        e = min(k + step, len(pick))
        bad = check_columns(ds.residues, ds.offsets, pick[k:e], ds.matrix, -11, -1, span[k:e], ops_h,
                            off_h[k:e + 1], n_h[k:e])
        assert not bad, {name: (len(v), pick[k + v[0]].tolist()) for name, v in bad.items()}
    sub = np.r_[0:200, len(pick) - 20:len(pick)]
    want, ospan = traceback_batch(ds.residues, ds.offsets, pick[sub], ds.matrix)
    assert np.array_equal(ospan, span[sub])
    got = [bytes(ops_h[off_h[p]:off_h[p] + n_h[p]]).decode() for p in sub]
    assert got == want


def test_errors(cm):
    ds = cmgen.family_dataset(2, [2, 2], lambda r: 80, 30, 200, 607)
    res = torch.from_numpy(ds.residues).cuda()
    off = torch.from_numpy(ds.offsets).cuda()
    pr = torch.from_numpy(np.array([[0, 1], [1, 0], [2, 3]], np.int32)).cuda()
    sc, ea, eb = cm.sw_score_batch(res, off, pr, ds.matrix, return_end=True)
    sa, sb = cm.sw_span_batch(res, off, pr, ds.matrix, sc, ea, eb, 0)
    cm.sync()
    assert (sc.cpu().numpy() > 0).all()
    # a column buffer one byte short for pair 1
    cap = ((ea - sa + 1) + (eb - sb + 1)).to(torch.int64)
    cap[1] -= 1
    op_off = torch.zeros(4, dtype=torch.int64, device="cuda")
    op_off[1:] = torch.cumsum(cap, 0)
    ops = torch.zeros(int(op_off[-1]), dtype=torch.uint8, device="cuda")
    n_ops = torch.zeros(3, dtype=torch.int32, device="cuda")
    import ctypes
    lib = cm._lib
    m = cm._matrix_host(ds.matrix)
    st = lib.cm_sw_traceback_batch(cm.context().handle, res.data_ptr(), off.data_ptr(), ds.n, pr.data_ptr(), 3,
                                   m.ctypes.data, -11, -1, sc.data_ptr(), ea.data_ptr(), eb.data_ptr(),
                                   sa.data_ptr(), sb.data_ptr(), op_off.data_ptr(), ops.data_ptr(),
                                   n_ops.data_ptr(), None)
    assert st == 0
    with pytest.raises(cm.CMError) as e:
        cm.sync()
    assert e.value.status == cm.CM_ERANGE
    n = n_ops.cpu().numpy()
    assert n[1] == -1 and n[0] > 0 and n[2] > 0
    # an end cell outside its sequence
    bad_ea = ea.clone()
    bad_ea[0] = 10000
    cm.sw_traceback_batch(res, off, pr, ds.matrix, sc, bad_ea, eb, sa, sb)
    with pytest.raises(cm.CMError) as e:
        cm.sync()
    assert e.value.status == cm.CM_ERANGE
    # gaps are validated on the host
    with pytest.raises(cm.CMError):
        cm.sw_traceback_batch(res, off, pr, ds.matrix, sc, ea, eb, sa, sb, -1, -3)
    del ctypes
