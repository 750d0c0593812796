"""Launch plans and the autotuner: every plan gives the oracle's exact results."""
import os

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


@pytest.fixture(scope="module")
def data():
    rng = np.random.default_rng(401)
    fam = cmgen.family_dataset(8, [6] * 8, lambda r: int(r.integers(20, 1400)), 1, 1600, 402)
    pool = cmgen.uniform_pool(30, 0, 900, 403)
    ds = cmgen.from_list([fam.seq(i) for i in range(fam.n)] + [pool.seq(i) for i in range(pool.n)])
    pairs = cmgen.random_pairs(rng, ds.n, 1200)
    ref = span_batch(ds.residues, ds.offsets, pairs, ds.matrix)
    return ds, pairs, ref


def run(cm, ctx, ds, pairs):
    res = torch.from_numpy(ds.residues).cuda()
    off = torch.from_numpy(ds.offsets).cuda()
    pr = torch.from_numpy(pairs).cuda()
    sc, ea, eb = cm.sw_score_batch(res, off, pr, ds.matrix, return_end=True, ctx=ctx)
    sa, sb = cm.sw_span_batch(res, off, pr, ds.matrix, sc, ea, eb, 0, ctx=ctx)
    s_only = cm.sw_score_batch(res, off, pr, ds.matrix, ctx=ctx)
    ctx.sync()
    out = np.stack([t.cpu().numpy() for t in (sc, ea, eb, sa, sb)], 1)
    return out, s_only.cpu().numpy()


@pytest.mark.parametrize("rmax", [8, 12, 16])
def test_every_plan_is_exact(cm, data, rmax):
    ds, pairs, ref = data
    ctx = cm.Context(0)
    for p in range(3):
        _, _, _ = ctx.get_plan(p)
    occ = [ctx.get_plan(p)[2] for p in range(3)]
    for bpc_pick in ("one", "max"):
        for p in range(3):
            ctx.set_plan(p, 16, 1)                      # occupancy limit of this rmax:
            ctx.set_plan(p, rmax, 1)
            mx = ctx.get_plan(p)[2]
            ctx.set_plan(p, rmax, 1 if bpc_pick == "one" else mx)
        out, s_only = run(cm, ctx, ds, pairs)
        bad = np.flatnonzero((out != ref).any(1))
        assert len(bad) == 0, (rmax, bpc_pick, pairs[bad[0]], out[bad[0]], ref[bad[0]])
        assert np.array_equal(s_only, ref[:, 0])
    assert all(o >= 1 for o in occ)
    ctx.close()


def test_autotune_and_plan_cache(cm, data, tmp_path):
    ds, pairs, ref = data
    ctx = cm.Context(0)
    res = torch.from_numpy(ds.residues).cuda()
    off = torch.from_numpy(ds.offsets).cuda()
    rows = ctx.autotune(res, off, torch.from_numpy(pairs).cuda(), ds.matrix, 0)
    assert len(rows) >= 3
    best = min(rows, key=lambda r: r[2])
    assert ctx.get_plan(0)[:2] == best[:2]
    out, s_only = run(cm, ctx, ds, pairs)
    assert np.array_equal(out, ref) and np.array_equal(s_only, ref[:, 0])
    path = str(tmp_path / "plans.txt")
    ctx.save_plans(path)
    ctx2 = cm.Context(0)
    ctx2.set_plan(0, 8, 1)
    ctx2.load_plans(path)
    assert ctx2.get_plan(0)[:2] == best[:2]
    bad = tmp_path / "bad.txt"
    bad.write_text("not a plan file\n")
    with pytest.raises(cm.CMError):
        ctx2.load_plans(str(bad))
    assert ctx2.get_plan(0)[:2] == best[:2]
    os.environ["CM_AUTOTUNE_CACHE"] = path
    try:
        ctx3 = cm.Context(0)
        assert ctx3.get_plan(0)[:2] == best[:2]
        os.environ["CM_AUTOTUNE_CACHE"] = str(bad)
        ctx4 = cm.Context(0)                      # corrupt cache: defaults
        assert ctx4.get_plan(0)[0] == 16
    finally:
        del os.environ["CM_AUTOTUNE_CACHE"]
    for c in (ctx, ctx2, ctx3, ctx4):
        c.close()
