"""cm_sw_score_batch_noalloc (the allocation-free score batch) against
cm_sw_score_batch: identical outputs on two calls in a row, the second with a
smaller input, for score-only and score+end calls; the limit is enforced."""
import ctypes

import numpy as np
import pytest

import cmgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1908_10574_amd as cm
    lib = cm.lib()
    P = ctypes.c_void_p
    lib.cm_sw_score_batch_noalloc.restype = ctypes.c_int32
    lib.cm_sw_score_batch_noalloc.argtypes = [P, P, P, ctypes.c_int32, P, ctypes.c_int64, P, ctypes.c_int32,
                                              ctypes.c_int32, P, P, P, P]
    return cm


def noalloc(cm, ctx, res, off, pairs, matrix, with_end):
    n = pairs.shape[0]
    sc = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    ea = torch.full((n,), -7, dtype=torch.int32, device="cuda") if with_end else None
    eb = torch.full((n,), -7, dtype=torch.int32, device="cuda") if with_end else None
    m = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32).reshape(-1))
    torch.cuda.current_stream().synchronize()
    st = cm.lib().cm_sw_score_batch_noalloc(ctx.handle, res.data_ptr(), off.data_ptr(), off.numel() - 1,
                                            pairs.data_ptr(), n, m.ctypes.data, -11, -1, sc.data_ptr(),
                                            ea.data_ptr() if with_end else None,
                                            eb.data_ptr() if with_end else None, None)
    return st, sc, ea, eb


def test_noalloc_matches_score_batch_two_calls(cm):
    ctx = cm.Context(0)
    big = cmgen.throughput_pool(n_pool=20000, n_pairs=1048576, seed=313)
    small = cmgen.allvsall_small()
    cases = [(big, big.pairs, False), (small, small.pairs[:3001], False),
             (big, big.pairs[:600000], True), (small, small.pairs[:2500], True)]
    for ds, pairs, with_end in cases:
        print("noalloc", len(pairs), "pairs, end cells" if with_end else "pairs, score only", flush=True)
        res = torch.from_numpy(ds.residues).cuda()
        off = torch.from_numpy(ds.offsets).cuda()
        pr = torch.from_numpy(np.ascontiguousarray(pairs)).cuda()
        st, sc, ea, eb = noalloc(cm, ctx, res, off, pr, ds.matrix, with_end)
        assert st == 0, cm.CMError(st)
        ref = cm.sw_score_batch(res, off, pr, ds.matrix, return_end=with_end, ctx=ctx)
        ctx.sync()
        if with_end:
            for a, b in zip((sc, ea, eb), ref):
                assert torch.equal(a, b)
        else:
            assert torch.equal(sc, ref)
        assert (sc.cpu().numpy() >= 0).all()
    ctx.close()


def test_noalloc_rejects_more_than_its_limit(cm):
    ctx = cm.Context(0)
    ds = cmgen.allvsall_small()
    res = torch.from_numpy(ds.residues).cuda()
    off = torch.from_numpy(ds.offsets).cuda()
    pr = torch.zeros((1048577, 2), dtype=torch.int32, device="cuda")
    st, sc, _, _ = noalloc(cm, ctx, res, off, pr, ds.matrix, False)
    assert st == cm.CM_EINVAL
    assert b"allocation-free limit" in cm.lib().cm_last_error()
    assert (sc.cpu().numpy() == -7).all()      # nothing was enqueued
    ctx.close()
