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


def test_adam_constant_gradient_closed_form():
    """Under a constant gradient g the bias-corrected moments are exactly g and
    g^2 at every step, so step t moves every weight by lr * g / (|g| + eps):
    after k steps w0 - k * lr * g / (|g| + eps).  A wrong bias correction at
    any step after the first breaks this."""
    rng = np.random.default_rng(6)
    w0 = rng.normal(size=200).astype(np.float32)
    g = (rng.normal(size=200) * 10.0 ** rng.integers(-3, 2, size=200)).astype(np.float32)
    w, m, v = w0.copy(), np.zeros(200, np.float32), np.zeros(200, np.float32)
    for t in range(1, 13):
        w, m, v = S.adam(w, g, m, v, t, lr=1e-3)
        want = w0.astype(np.float64) - t * 1e-3 * g / (np.abs(g.astype(np.float64)) + 1e-8)
        assert np.allclose(w, want, atol=2e-6, rtol=0), (t, np.abs(w - want).max())


def test_adam_second_step_after_a_zero_gradient():
    """g at step 1, zero at step 2.  The moments after step 2 are b1(1-b1)g and
    b2(1-b2)g^2; divided by 1-b1^2 = (1-b1)(1+b1) and 1-b2^2 they become
    g b1/(1+b1) and g^2 b2/(1+b2), so the second move is
    lr * b1/(1+b1) * sqrt((1+b2)/b2) * sign(g) = 6.7006e-4 * sign(g) at the
    defaults (eps negligible for |g| ~ 1)."""
    rng = np.random.default_rng(7)
    w0 = rng.normal(size=64).astype(np.float32)
    g = rng.choice([-1.0, 1.0], size=64).astype(np.float32) * rng.uniform(0.5, 2.0, size=64).astype(np.float32)
    z = np.zeros(64, np.float32)
    w1, m, v = S.adam(w0, g, z, z, 1, lr=1e-3)
    w2, m, v = S.adam(w1, np.zeros(64, np.float32), m, v, 2, lr=1e-3)
    move = 1e-3 * (0.9 / 1.9) * np.sqrt(1.999 / 0.999)
    assert abs(move - 6.7006e-4) < 1e-8
    assert np.allclose(w1 - w2, move * np.sign(g), atol=2e-7)


def test_adam_is_invariant_to_gradient_scale():
    """Adam divides the first moment by the root of the second, so scaling every
    gradient by c > 0 leaves the trajectory unchanged (while eps is negligible);
    a moment that mixes g and g^2 wrongly would not be."""
    rng = np.random.default_rng(8)
    w0 = rng.normal(size=128).astype(np.float32)
    gs = [rng.normal(size=128).astype(np.float32) for _ in range(6)]
    traj = []
    for c in (1.0, 1000.0):
        w, m, v = w0.copy(), np.zeros(128, np.float32), np.zeros(128, np.float32)
        for t, g in enumerate(gs, 1):
            w, m, v = S.adam(w, (g * c).astype(np.float32), m, v, t, lr=1e-3)
        traj.append(w)
    assert np.allclose(traj[0], traj[1], atol=1e-6)
    assert np.abs(traj[0] - w0).max() > 1e-3
