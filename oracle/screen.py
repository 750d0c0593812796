"""CPU reference of the learned pair screen.  Test infrastructure only.

The screen is not in the paper: it is a learned pre-filter placed in front of
the exact similarity function f of Section 4 (which still decides every
pair it lets through).  Its definition here:

* features: for every protein, the counts of its 3-mers hashed into 1,024
  buckets (code = 400*a_p + 20*a_{p+1} + a_{p+2}; bucket = the top 10 bits of
  the 32-bit product code * 2654435761), divided by 8 and rounded to bf16;
* pair input: x = [|c_a - c_b|, c_a * c_b] (2,048 values), computed in fp32
  from the bf16 counts, rounded to bf16;
* network: z = W3 relu(W2 relu(W1 x + b1) + b2) + b3 with bf16 weights, fp32
  accumulation, hidden activations rounded to bf16 (512 and 512 units);
* loss: binary cross-entropy on logits, max(z,0) - z*y + log1p(exp(-|z|)),
  averaged over the batch; labels y = [Smith-Waterman score >= T];
* optimizer: Adam on fp32 master weights (bf16 copies used by the network).

Rounding to bf16 is round-to-nearest-even on the fp32 bit pattern.
"""
from __future__ import annotations

import numpy as np

N_BUCKETS = 1024
HIDDEN = 512
N_IN = 2 * N_BUCKETS
HASH_MUL = 2654435761


# ---------------------------------------------------------------------------
# bf16
# ---------------------------------------------------------------------------
def bf16_bits(x) -> np.ndarray:
    """fp32 -> bf16 bit patterns (uint16), round to nearest even."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def bf16_round(x) -> np.ndarray:
    return bf16_value(bf16_bits(x))


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------
def kmer_counts(seq) -> np.ndarray:
    """1,024 hashed 3-mer counts of one protein (int64)."""
    s = np.asarray(seq, dtype=np.int64)
    out = np.zeros(N_BUCKETS, dtype=np.int64)
    if len(s) < 3:
        return out
    code = 400 * s[:-2] + 20 * s[1:-1] + s[2:]
    bucket = ((code * HASH_MUL) & 0xFFFFFFFF) >> 22
    np.add.at(out, bucket, 1)
    return out


def features(residues, offsets) -> np.ndarray:
    """bf16 bit patterns [n][1024] of count/8."""
    n = len(offsets) - 1
    out = np.zeros((n, N_BUCKETS), dtype=np.uint16)
    for i in range(n):
        c = kmer_counts(residues[offsets[i]:offsets[i + 1]])
        out[i] = bf16_bits(c.astype(np.float32) / np.float32(8.0))
    return out


def pair_input(feat_bits, pairs) -> np.ndarray:
    """bf16-rounded fp32 inputs [P][2048] for pair rows (a, b)."""
    fa = bf16_value(feat_bits[pairs[:, 0]])
    fb = bf16_value(feat_bits[pairs[:, 1]])
    x = np.concatenate([np.abs(fa - fb), fa * fb], axis=1).astype(np.float32)
    return bf16_round(x)


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
SHAPES = [("W1", (HIDDEN, N_IN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("W3", (1, HIDDEN)), ("b3", (1,))]


def n_params(shapes=SHAPES) -> int:
    return int(sum(np.prod(s) for _, s in shapes))


def unflatten(flat, shapes=SHAPES) -> dict:
    out, k = {}, 0
    for name, shp in shapes:
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[k:k + n]).reshape(shp)
        k += n
    return out


def flatten(params, shapes=SHAPES) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).reshape(-1) for name, _ in shapes])


def init_params(seed: int, shapes=SHAPES) -> np.ndarray:
    """Kaiming-uniform weights (bound sqrt(6/fan_in)), zero biases, as one fp32 vector."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in shapes:
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shp[1])
            parts.append(rng.uniform(-bound, bound, size=shp).astype(np.float32).reshape(-1))
        else:
            parts.append(np.zeros(int(np.prod(shp)), np.float32))
    return np.concatenate(parts)


def forward(flat_master, x, rounding=True, shapes=SHAPES):
    """Logits and the activations the backward pass needs.

    With rounding, weights are the bf16 copies of the fp32 master and hidden
    activations are rounded to bf16; accumulation is fp64 here (the GPU
    accumulates in fp32, a difference far below the test tolerance).
    """
    p = unflatten(np.asarray(flat_master, dtype=np.float32 if rounding else np.float64), shapes)
    rnd = bf16_round if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    W1, W2, W3 = (rnd(p[k]).astype(np.float64) for k in ("W1", "W2", "W3"))
    b1, b2, b3 = (p[k].astype(np.float64) for k in ("b1", "b2", "b3"))
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ W1.T + b1
    h1 = rnd(np.maximum(a1, 0).astype(np.float32) if rounding else np.maximum(a1, 0)).astype(np.float64)
    a2 = h1 @ W2.T + b2
    h2 = rnd(np.maximum(a2, 0).astype(np.float32) if rounding else np.maximum(a2, 0)).astype(np.float64)
    z = (h2 @ W3.T + b3)[:, 0]
    return z, dict(x=x, h1=h1, h2=h2, W2=W2, W3=W3)


def bce(z, y) -> float:
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def backward(z, y, cache, shapes=SHAPES) -> np.ndarray:
    """Gradient of the mean BCE with respect to every master parameter (flat)."""
    n = len(z)
    y = np.asarray(y, dtype=np.float64)
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n                      # [n]
    h1, h2, x = cache["h1"], cache["h2"], cache["x"]
    gW3 = (dz[:, None] * h2).sum(0)[None, :]
    gb3 = np.array([dz.sum()])
    dh2 = dz[:, None] * cache["W3"][0][None, :] * (h2 > 0)       # [n][512]
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ cache["W2"]) * (h1 > 0)
    gW1 = dh1.T @ x
    gb1 = dh1.sum(0)
    g = dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2, W3=gW3, b3=gb3)
    return flatten(g, shapes)


def adam(master, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (master, m, v) in fp32."""
    g = np.asarray(grad, dtype=np.float32)
    m = (beta1 * m + (1 - beta1) * g).astype(np.float32)
    v = (beta2 * v + (1 - beta2) * g * g).astype(np.float32)
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    master = (master - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
    return master, m, v
