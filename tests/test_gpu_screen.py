"""GPU screen (features, bf16-MFMA MLP forward/backward, Adam) vs the CPU reference.

Weights are drawn on the CPU (oracle.screen.init_params) and loaded into the
GPU screen, so neither side's inputs come from the other.
"""
import numpy as np
import pytest

import cmgen
from oracle import screen as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cm():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1908_10574_amd as cm
    return cm


@pytest.fixture(scope="module")
def data(cm):
    ds = cmgen.allvsall_small()
    res = torch.from_numpy(ds.residues).cuda()
    off = torch.from_numpy(ds.offsets).cuda()
    feat = cm.kmer_features(res, off)
    cm.sync()
    return ds, res, off, feat


def feat_bits(feat):
    return feat.view(torch.int16).cpu().numpy().view(np.uint16)


def test_features_bit_exact(cm, data):
    ds, res, off, feat = data
    assert np.array_equal(feat_bits(feat), S.features(ds.residues, ds.offsets))
    long = cmgen.uniform_pool(40, 0, 5000, 9)
    f2 = cm.kmer_features(torch.from_numpy(long.residues).cuda(), torch.from_numpy(long.offsets).cuda())
    cm.sync()
    assert np.array_equal(feat_bits(f2), S.features(long.residues, long.offsets))


def test_logits_within_tolerance(cm, data):
    ds, res, off, feat = data
    w = S.init_params(11)
    scr = cm.Screen(0)
    scr.set_weights(w)
    m, b = scr.get_weights()
    assert np.array_equal(m, w)
    assert np.array_equal(b[:512 * 2048], S.bf16_bits(w[:512 * 2048]))
    rng = np.random.default_rng(12)
    pairs = cmgen.random_pairs(rng, ds.n, 777)
    z = scr.infer(feat, torch.from_numpy(pairs).cuda()).cpu().numpy()
    zr, _ = S.forward(w, S.pair_input(feat_bits(feat), pairs))
    err = np.abs(z - zr).max()
    assert err < 2e-2, err
    print("max |logit diff|", err, "logit std", zr.std())


def _batch(ds, n, seed):
    from oracle import sw_batch
    rng = np.random.default_rng(seed)
    fam_pairs = []
    for _ in range(n // 2):
        f = rng.integers(0, 10)
        idx = np.flatnonzero(ds.family == f)
        a, b = rng.choice(idx, 2, replace=False)
        fam_pairs.append((a, b))
    pairs = np.concatenate([np.array(fam_pairs), cmgen.random_pairs(rng, ds.n, n - n // 2)]).astype(np.int32)
    y = (sw_batch(ds.residues, ds.offsets, pairs, ds.matrix, with_end=False) >= 120).astype(np.uint8)
    return pairs, y


def test_gradients_match_reference(cm, data):
    ds, res, off, feat = data
    w = S.init_params(13)
    scr = cm.Screen(0)
    scr.set_weights(w)
    # the second batch, larger and ragged, makes the same screen grow its workspace
    for n, seed in ((300, 14), (1000, 17)):
        pairs, y = _batch(ds, n, seed)
        g, loss = scr.grads(feat, torch.from_numpy(pairs).cuda(), torch.from_numpy(y).cuda())
        z, cache = S.forward(w, S.pair_input(feat_bits(feat), pairs))
        gr = S.backward(z, y, cache)
        assert abs(loss - S.bce(z, y)) < 1e-3
        gp, rp = S.unflatten(g), S.unflatten(gr)
        for name, _ in S.SHAPES:
            rel = np.linalg.norm(gp[name] - rp[name]) / max(np.linalg.norm(rp[name]), 1e-30)
            assert rel < 1e-2, (n, name, rel)


def test_training_reduces_loss_and_adam_matches(cm, data):
    ds, res, off, feat = data
    w = S.init_params(15)
    scr = cm.Screen(0)
    scr.set_weights(w)
    pairs, y = _batch(ds, 512, 16)
    tp, ty = torch.from_numpy(pairs).cuda(), torch.from_numpy(y).cuda()
    # four Adam steps, each compared with the reference update from the same
    # gradient (the GPU's gradient is deterministic, so grads() before a step
    # returns the gradient that step uses)
    want, m, v = w.copy(), np.zeros_like(w), np.zeros_like(w)
    first = None
    for t in range(1, 5):
        g, _ = scr.grads(feat, tp, ty)
        loss = scr.train_step(feat, tp, ty, lr=1e-3)
        first = loss if first is None else first
        got, _ = scr.get_weights()
        want, m, v = S.adam(want, g, m, v, t, lr=1e-3)
        assert np.abs(got - want).max() < 1e-6, (t, np.abs(got - want).max())
        want = got   # next step starts from the GPU's weights
    losses = [scr.train_step(feat, tp, ty, lr=1e-3) for _ in range(40)]
    assert losses[-1] < 0.5 * first, (first, losses[-1])


def test_training_run_equals_steps(cm, data):
    """cm_screen_train over the given order equals cm_screen_train_step over the
    same batches bit for bit (weights), with a ragged last batch; its loss log
    holds each step's mean loss before the update."""
    ds, res, off, feat = data
    w = S.init_params(21)
    pairs, y = _batch(ds, 1000, 22)
    tp, ty = torch.from_numpy(pairs).cuda(), torch.from_numpy(y).cuda()
    a = cm.Screen(0)
    a.set_weights(w)
    log = a.train(feat, tp, ty, epochs=2, batch=384, lr=2e-3, shuffle=False, drop_last=False)
    assert len(log) == 2 * 3
    b = cm.Screen(0)
    b.set_weights(w)
    want = []
    for _ in range(2):
        for k in range(0, 1000, 384):
            want.append(b.train_step(feat, tp[k:k + 384], ty[k:k + 384], lr=2e-3))
    wa, ba = a.get_weights()
    wb, bb = b.get_weights()
    assert np.array_equal(wa, wb) and np.array_equal(ba, bb)
    assert np.allclose(log, want, rtol=1e-5, atol=1e-7), (log, want)
    # the first step's loss is the reference loss of the initial weights
    z, _ = S.forward(w, S.pair_input(feat_bits(feat), pairs[:384]))
    assert abs(log[0] - S.bce(z, y[:384])) < 1e-3


def test_training_run_shuffles_and_learns(cm, data):
    ds, res, off, feat = data
    pairs, y = _batch(ds, 4000, 23)
    tp, ty = torch.from_numpy(pairs).cuda(), torch.from_numpy(y).cuda()
    runs = []
    for seed in (5, 5, 6):
        scr = cm.Screen(3)
        log = scr.train(feat, tp, ty, epochs=4, batch=256, lr=1e-3, seed=seed)
        runs.append((log, scr.get_weights()[0]))
    assert len(runs[0][0]) == 4 * (4000 // 256)
    assert np.array_equal(runs[0][1], runs[1][1])          # same seed, same run
    assert not np.array_equal(runs[0][1], runs[2][1])      # another order
    log = runs[0][0]
    assert log[-15:].mean() < 0.7 * log[:15].mean()
    with pytest.raises(cm.CMError):
        cm.Screen(0).train(feat, tp, ty, epochs=1, batch=1 << 21, drop_last=False)


def test_save_load_roundtrip(cm, data, tmp_path):
    ds, res, off, feat = data
    scr = cm.Screen(7)
    pairs = torch.from_numpy(cmgen.random_pairs(np.random.default_rng(1), ds.n, 100)).cuda()
    z1 = scr.infer(feat, pairs).cpu().numpy()
    p = tmp_path / "s.bin"
    scr.save(str(p))
    s2 = cm.Screen.load(str(p))
    z2 = s2.infer(feat, pairs).cpu().numpy()
    assert np.array_equal(z1, z2)


def test_trained_screen_quality_and_screened_recall(cm):
    """Train on GPU-labelled pairs of one family set; screen ClusterMerge on another."""
    from paper_1908_10574_amd import screen_train as st
    ds = cmgen.screen_training(seed=404, n_seqs=4000, n_families=400, n_pairs=200000)
    scr, tau, info = st.train_on_dataset(ds, epochs=3, seed=3)
    print(info)
    assert info["loss_per_epoch"][-1] < info["loss_per_epoch"][0]
    assert info["holdout_auc"] > 0.97
    assert info["holdout_pos_kept"] >= 0.99
    test = cmgen.clustermerge_families(n_seqs=2000, n_families=200, seed=222)
    res, off = torch.from_numpy(test.residues).cuda(), torch.from_numpy(test.offsets).cuda()
    plain = cm.clustermerge_run(res, off, test.matrix)
    # the size guard the benchmark uses: representative pairs of clusters whose
    # member counts multiply to 64 or more bypass the screen
    scr_run = cm.clustermerge_run(res, off, test.matrix, screen=scr, screen_tau=tau, screen_min_product=64)
    ps, ss = plain["stats"], scr_run["stats"]
    print({k: (ps[k], ss[k]) for k in ("n_similar_pairs", "aligned_pairs", "aligned_cells", "screened_out",
                                      "t_total_s")})
    assert ss["screened_out"] > 0
    assert ss["aligned_cells"] < ps["aligned_cells"]
    assert ss["n_similar_pairs"] >= 0.995 * ps["n_similar_pairs"]
    # screened output is still exact: every reported pair is a true similar pair
    found = {(int(x), int(y)) for x, y in plain["pairs"]}
    assert all((int(x), int(y)) in found for x, y in scr_run["pairs"][:: max(1, len(scr_run["pairs"]) // 5000)])
