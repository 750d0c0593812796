"""Pins for the CPU reference of the learned screen (CPU only).

bf16 rounding is checked against torch's own float->bfloat16 conversion; the
3-mer featurizer against a dictionary count; the backward pass against fp64
central finite differences of the loss on a small network; Adam against the
first-step closed form (the first update of every weight is lr * sign(g)).
"""
import numpy as np
import torch

import cmgen
from oracle import screen as S

TINY = [("W1", (8, 16)), ("b1", (8,)), ("W2", (8, 8)), ("b2", (8,)), ("W3", (1, 8)), ("b3", (1,))]


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.normal(0, 1e-3, 1000),
                        [0.0, 1.0, -1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 255.0, 256.0, 257.0, 3.0e38]]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(S.bf16_bits(x), want)
    assert np.array_equal(S.bf16_value(S.bf16_bits(x)), torch.from_numpy(x).to(torch.bfloat16).float().numpy())


def test_kmer_counts_by_dictionary():
    rng = np.random.default_rng(2)
    for L in (0, 1, 2, 3, 10, 400):
        s = rng.integers(0, 20, size=L)
        want = np.zeros(1024, np.int64)
        for p in range(L - 2):
            code = 400 * int(s[p]) + 20 * int(s[p + 1]) + int(s[p + 2])
            want[((code * 2654435761) % 2 ** 32) // 2 ** 22] += 1
        got = S.kmer_counts(s)
        assert np.array_equal(got, want)
        assert got.sum() == max(0, L - 2)


def test_features_small_counts_exact():
    ds = cmgen.allvsall_small()
    f = S.features(ds.residues, ds.offsets)
    for i in (0, 5, 99):
        c = S.kmer_counts(ds.seq(i))
        assert np.array_equal(S.bf16_value(f[i]), (c / 8.0).astype(np.float32))   # counts <= 256: exact


def test_pair_input_symmetric():
    ds = cmgen.allvsall_small()
    f = S.features(ds.residues, ds.offsets)
    p = np.array([[1, 2], [3, 7]])
    assert np.array_equal(S.pair_input(f, p), S.pair_input(f, p[:, ::-1]))


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    w = S.init_params(4, TINY).astype(np.float64)
    w[8 * 16:8 * 16 + 8] = rng.normal(0, 0.1, 8)          # nonzero b1
    x = np.abs(rng.normal(0, 1, size=(12, 16)))
    y = (rng.random(12) < 0.5).astype(np.float64)
    z, cache = S.forward(w, x, rounding=False, shapes=TINY)
    g = S.backward(z, y, cache, shapes=TINY)
    h = 1e-6
    num = np.zeros_like(w)
    for k in range(len(w)):
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        num[k] = (S.bce(S.forward(wp, x, False, TINY)[0], y) - S.bce(S.forward(wm, x, False, TINY)[0], y)) / (2 * h)
    assert np.allclose(g, num, rtol=1e-5, atol=1e-8), np.abs(g - num).max()


def test_bce_stable_form():
    z = np.linspace(-20, 20, 81)
    for y in (0.0, 1.0):
        naive = np.mean(-(y * np.log(1 / (1 + np.exp(-z))) + (1 - y) * np.log(1 - 1 / (1 + np.exp(-z)))))
        assert abs(S.bce(z, np.full_like(z, y)) - naive) < 1e-6


def test_adam_first_step_is_sign():
    rng = np.random.default_rng(5)
    w = rng.normal(size=100).astype(np.float32)
    g = rng.normal(size=100).astype(np.float32)
    w1, m, v = S.adam(w, g, np.zeros(100, np.float32), np.zeros(100, np.float32), 1, lr=1e-3)
    assert np.allclose(w1, w - 1e-3 * np.sign(g), atol=1e-7)


def test_init_bounds():
    w = S.init_params(0)
    p = S.unflatten(w)
    assert len(w) == S.n_params() == 1312257
    assert np.abs(p["W1"]).max() <= np.sqrt(6 / 2048) and np.abs(p["W2"]).max() <= np.sqrt(6 / 512)
    assert (p["b1"] == 0).all() and (p["b3"] == 0).all()
