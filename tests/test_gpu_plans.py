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


PLANS = [(0, 8), (0, 12), (0, 16), (1, 4), (1, 8), (2, 32)]


@pytest.mark.parametrize("packed,rmax", PLANS)
def test_every_plan_is_exact(cm, data, packed, rmax):
    """Every (kernel, rows-per-lane limit, blocks per CU) gives the oracle's results;
    the packed kernel serves the score pass, the others keep an int32 plan."""
    ds, pairs, ref = data
    ctx = cm.Context(0)
    assert ctx.get_plan(0)[:2] == (2, 32)           # default score plan: shared-query packed
    for bpc_pick in ("one", "max"):
        for p in range(3):
            if packed and p != 0:
                ctx.set_plan(p, 0, 16, 1)
                continue
            ctx.set_plan(p, packed, rmax, 1)
            mx = ctx.get_plan(p)[3]
            assert mx >= 1
            ctx.set_plan(p, packed, rmax, 1 if bpc_pick == "one" else mx)
        out, s_only = run(cm, ctx, ds, pairs)
        bad = np.flatnonzero((out != ref).any(1))
        assert len(bad) == 0, (packed, rmax, bpc_pick, pairs[bad[0]], out[bad[0]], ref[bad[0]])
        assert np.array_equal(s_only, ref[:, 0])
    with pytest.raises(cm.CMError):
        ctx.set_plan(1, 1, 8, 1)                     # packed plans exist for the score pass only
    with pytest.raises(cm.CMError):
        ctx.set_plan(0, 1, 16, 1)                    # packed rows-per-lane limit is 4 or 8
    with pytest.raises(cm.CMError):
        ctx.set_plan(0, 2, 16, 1)                    # the shared-query kernel takes up to 32 rows
    ctx.close()


def test_autotune_and_plan_cache(cm, data, tmp_path):
    ds, pairs, ref = data
    ctx = cm.Context(0)
    res = torch.from_numpy(ds.residues).cuda()
    off = torch.from_numpy(ds.offsets).cuda()
    rows = ctx.autotune(res, off, torch.from_numpy(pairs).cuda(), ds.matrix, 0)
    assert len(rows) >= 6 and {r[0] for r in rows} == {0, 1, 2}
    best = min(rows, key=lambda r: r[3])
    assert ctx.get_plan(0)[:3] == best[:3]
    out, s_only = run(cm, ctx, ds, pairs)
    assert np.array_equal(out, ref) and np.array_equal(s_only, ref[:, 0])
    path = str(tmp_path / "plans.txt")
    ctx.save_plans(path)
    ctx2 = cm.Context(0)
    ctx2.set_plan(0, 0, 8, 1)
    ctx2.load_plans(path)
    assert ctx2.get_plan(0)[:3] == best[:3]
    bad = tmp_path / "bad.txt"
    bad.write_text("not a plan file\n")
    with pytest.raises(cm.CMError):
        ctx2.load_plans(str(bad))
    assert ctx2.get_plan(0)[:3] == best[:3]
    os.environ["CM_AUTOTUNE_CACHE"] = path
    try:
        ctx3 = cm.Context(0)
        assert ctx3.get_plan(0)[:3] == best[:3]
        os.environ["CM_AUTOTUNE_CACHE"] = str(bad)
        ctx4 = cm.Context(0)                      # corrupt cache: defaults
        assert ctx4.get_plan(0)[:2] == (2, 32) and ctx4.get_plan(1)[:2] == (0, 16)
    finally:
        del os.environ["CM_AUTOTUNE_CACHE"]
    for c in (ctx, ctx2, ctx3, ctx4):
        c.close()
