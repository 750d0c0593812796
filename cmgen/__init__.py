"""Seeded synthetic protein-family generator.

This module produces INPUTS only: residue codes, offsets, family labels, a
substitution matrix and pair lists.  It contains none of the alignment or
clustering arithmetic, so both the CPU oracle tests and the GPU path can draw
their inputs from it without sharing any of the method's code.

The paper evaluates on real genomes (Section 6: the OMA 13-bacteria 59K set, the
QfO 90K set, a Streptococcus set) and scores with PAM250 (Section 4); none of
these are available here.  The synthetic families below stand in for them:

* alphabet: the 20 standard amino acids ``ACDEFGHIKLMNPQRSTVWY`` coded 0..19,
  one byte per residue, concatenated, with int64 offsets (the paper's
  replicated dataset indexed by 4-byte sequence ids, Section 5.3);
* background: i.i.d. uniform residue frequencies;
* substitution matrix: symmetric, diagonal uniform in 4..11, off-diagonal in
  -4..3 drawn from a skewed pmf (mean about -2.4) so that unrelated sequences
  score far below the similarity threshold 120;
* family member: an independent mutation of a random ancestor, with a 30%
  substitution rate and a 5% per-position indel event rate (50/50 insertion or
  deletion, geometric length with mean 3);
* family sizes: rank-size Zipf (size of family k proportional to k**-1.2);
* lengths: uniform or lognormal as the workload states, clipped to its range.

Every random draw comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

ALPHABET = "ACDEFGHIKLMNPQRSTVWY"
N_RES = 20

#: off-diagonal substitution values -4..3 and their probabilities
OFFDIAG_VALUES = np.arange(-4, 4, dtype=np.int64)
OFFDIAG_PMF = np.array([0.35, 0.25, 0.15, 0.10, 0.06, 0.04, 0.03, 0.02])
MATRIX_SEED = 1917   # first seed >= 1908 passing the calibration gate (tests/golden/matrix_gate.py)

GAP_OPEN = -11      # a gap of length k costs GAP_OPEN + (k-1)*GAP_EXTEND
GAP_EXTEND = -1
THRESHOLD = 120     # similar pair: score >= 120
FULL_MERGE_T = 166  # mT at this scale (the paper's 250/181 ratio applied to 120)
MAX_UNCOVERED = 15  # mU (Section 6.1)


def encode(text: str) -> np.ndarray:
    """Letters -> residue codes (uint8)."""
    lut = {c: i for i, c in enumerate(ALPHABET)}
    return np.array([lut[c] for c in text], dtype=np.uint8)


def decode(codes) -> str:
    return "".join(ALPHABET[int(c)] for c in codes)


def make_matrix(seed: int = MATRIX_SEED) -> np.ndarray:
    """Symmetric 20x20 int32 substitution matrix.

    Diagonal uniform on 4..11; each upper-triangle off-diagonal entry drawn from
    ``OFFDIAG_PMF`` over -4..3 and mirrored.
    """
    rng = np.random.default_rng(seed)
    m = np.zeros((N_RES, N_RES), dtype=np.int32)
    diag = rng.integers(4, 12, size=N_RES)
    iu = np.triu_indices(N_RES, k=1)
    off = rng.choice(OFFDIAG_VALUES, size=len(iu[0]), p=OFFDIAG_PMF)
    m[iu] = off
    m = m + m.T
    m[np.arange(N_RES), np.arange(N_RES)] = diag
    return m.astype(np.int32)


def background() -> np.ndarray:
    return np.full(N_RES, 1.0 / N_RES)


def random_residues(rng, n: int) -> np.ndarray:
    return rng.integers(0, N_RES, size=n, dtype=np.uint8)


def mutate(rng, anc: np.ndarray, sub_rate=0.30, indel_rate=0.05, geo_p=1.0 / 3.0) -> np.ndarray:
    """One family member from its ancestor.

    Per ancestor position: substitution with probability ``sub_rate`` (a
    background residue other than the original); independently an indel event
    with probability ``indel_rate``: half are insertions of k ~ Geometric(geo_p)
    background residues after the position, half deletions of k residues
    starting at (and including) the position.
    """
    L = len(anc)
    seq = anc.copy()
    sub = rng.random(L) < sub_rate
    r = rng.integers(0, N_RES - 1, size=L, dtype=np.int64)
    r = np.where(r >= seq, r + 1, r)                     # uniform over the 19 others
    seq = np.where(sub, r, seq).astype(np.uint8)
    ev = np.flatnonzero(rng.random(L) < indel_rate)
    if len(ev) == 0:
        return seq
    is_ins = rng.random(len(ev)) < 0.5
    klen = rng.geometric(geo_p, size=len(ev))
    keep = np.ones(L, dtype=bool)
    inserts = []
    for p, ins, k in zip(ev, is_ins, klen):
        if ins:
            inserts.append((p, random_residues(rng, int(k))))
        elif keep[p]:
            keep[p:p + k] = False
    if not inserts:
        return seq[keep]
    pieces, prev = [], 0
    for p, res in inserts:
        seg = seq[prev:p + 1]
        pieces.append(seg[keep[prev:p + 1]])
        pieces.append(res)
        prev = p + 1
    seg = seq[prev:]
    pieces.append(seg[keep[prev:]])
    return np.concatenate(pieces).astype(np.uint8)


def clip(rng, seq: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """Truncate the tail above ``hi``; pad with background residues below ``lo``."""
    if len(seq) > hi:
        return seq[:hi]
    if len(seq) < lo:
        return np.concatenate([seq, random_residues(rng, lo - len(seq))])
    return seq


def zipf_sizes(n_seqs: int, n_families: int, s: float = 1.2) -> np.ndarray:
    """Rank-size Zipf family sizes: n_k proportional to k**-s, each >= 1, summing to n_seqs.

    Largest-remainder rounding on the part above the floor of one member.
    """
    w = np.arange(1, n_families + 1, dtype=np.float64) ** -s
    extra = n_seqs - n_families
    raw = w / w.sum() * extra
    base = np.floor(raw).astype(np.int64)
    rem = extra - base.sum()
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:rem]] += 1
    return base + 1


@dataclass
class Dataset:
    residues: np.ndarray          # uint8, concatenated codes 0..19
    offsets: np.ndarray           # int64, n+1
    family: np.ndarray            # int32 family id per sequence (-1: none)
    matrix: np.ndarray            # int32 [20][20]
    pairs: np.ndarray | None = None   # int32 [P][2] (a, b), optional
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def seq(self, i: int) -> np.ndarray:
        return self.residues[self.offsets[i]:self.offsets[i + 1]]


def _pack(seqs, fam, matrix, meta, pairs=None) -> Dataset:
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    offsets = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    res = np.concatenate(seqs).astype(np.uint8) if len(seqs) else np.zeros(0, np.uint8)
    return Dataset(res, offsets, np.asarray(fam, dtype=np.int32), matrix, pairs, meta)


def family_dataset(n_families: int, sizes, length_fn, lo: int, hi: int, seed: int,
                   matrix_seed: int = MATRIX_SEED, sub_rate: float = 0.30,
                   indel_rate: float = 0.05) -> Dataset:
    """Families of mutated copies of random ancestors, shuffled by the seed
    (member divergence: substitution and indel rates of ``mutate``)."""
    rng = np.random.default_rng(seed)
    seqs, fam = [], []
    for f in range(n_families):
        L = int(np.clip(length_fn(rng), lo, hi))
        anc = random_residues(rng, L)
        for _ in range(int(sizes[f])):
            seqs.append(clip(rng, mutate(rng, anc, sub_rate, indel_rate), lo, hi))
            fam.append(f)
    perm = rng.permutation(len(seqs))
    seqs = [seqs[i] for i in perm]
    fam = np.asarray(fam, dtype=np.int32)[perm]
    meta = dict(seed=seed, matrix_seed=matrix_seed, n_families=n_families, lo=lo, hi=hi,
                sub_rate=sub_rate, indel_rate=indel_rate)
    return _pack(seqs, fam, make_matrix(matrix_seed), meta)


def lognormal_len(median: float, sigma: float):
    mu = np.log(median)
    return lambda rng: int(round(rng.lognormal(mu, sigma)))


def all_pairs(n: int) -> np.ndarray:
    """Every (a, b) with a < b, row-major."""
    a, b = np.triu_indices(n, k=1)
    return np.stack([a, b], axis=1).astype(np.int32)


# ---------------------------------------------------------------------------
# The five workloads.  Each returns a Dataset; sizes follow the workload text.
# ---------------------------------------------------------------------------

def allvsall_small(seed: int = 101) -> Dataset:
    """100 proteins = 10 families x 10, ancestor length U[50,400], all 4,950 pairs."""
    ds = family_dataset(10, [10] * 10, lambda rng: int(rng.integers(50, 401)), 50, 400, seed)
    ds.pairs = all_pairs(ds.n)
    ds.meta["workload"] = "allvsall-100"
    return ds


def clustermerge_families(n_seqs: int = 20000, n_families: int = 2000, seed: int = 202,
                          median: float = 350.0, sigma: float = 0.6, lo: int = 30,
                          hi: int = 2000, sub_rate: float = 0.30, indel_rate: float = 0.05) -> Dataset:
    """Zipf(1.2) families, lognormal lengths (median 350, sigma 0.6) clipped to [lo, hi]."""
    sizes = zipf_sizes(n_seqs, n_families)
    ds = family_dataset(n_families, sizes, lognormal_len(median, sigma), lo, hi, seed,
                        sub_rate=sub_rate, indel_rate=indel_rate)
    ds.meta.update(workload=f"clustermerge-{n_seqs}", median=median, sigma=sigma)
    return ds


def throughput_pool(n_pool: int = 200000, n_pairs: int = 1000000, seed: int = 303,
                    long_frac: float = 0.2, lo: int = 30, hi: int = 5000) -> Dataset:
    """Random pool: 80% lognormal(median 300, sigma 0.6), 20% U[1000,5000]; random a != b pairs."""
    rng = np.random.default_rng(seed)
    is_long = rng.random(n_pool) < long_frac
    short = np.rint(rng.lognormal(np.log(300.0), 0.6, size=n_pool)).astype(np.int64)
    longl = rng.integers(1000, 5001, size=n_pool)
    lens = np.clip(np.where(is_long, longl, short), lo, hi)
    offsets = np.zeros(n_pool + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    res = rng.integers(0, N_RES, size=int(offsets[-1]), dtype=np.uint8)
    a = rng.integers(0, n_pool, size=n_pairs)
    b = rng.integers(0, n_pool - 1, size=n_pairs)
    b = np.where(b >= a, b + 1, b)
    pairs = np.stack([a, b], axis=1).astype(np.int32)
    meta = dict(seed=seed, workload=f"throughput-{n_pairs}", n_pool=n_pool, lo=lo, hi=hi)
    return Dataset(res, offsets, np.full(n_pool, -1, np.int32), make_matrix(), pairs, meta)


def screen_training(seed: int = 404, n_seqs: int = 20000, n_families: int = 2000,
                    n_pairs: int = 2000000, within_frac: float = 0.5) -> Dataset:
    """Separate family dataset plus training pairs: half within-family, half uniform."""
    ds = clustermerge_families(n_seqs, n_families, seed)
    rng = np.random.default_rng(seed + 1)
    n_in = int(n_pairs * within_frac)
    order = np.argsort(ds.family, kind="stable")
    fam_sorted = ds.family[order]
    starts = np.searchsorted(fam_sorted, np.arange(n_families))
    ends = np.searchsorted(fam_sorted, np.arange(n_families), side="right")
    sizes = ends - starts
    multi = np.flatnonzero(sizes >= 2)
    w = sizes[multi].astype(np.float64) ** 2
    f = rng.choice(multi, size=n_in, p=w / w.sum())
    i = rng.integers(0, sizes[f])
    j = rng.integers(0, sizes[f] - 1)
    j = np.where(j >= i, j + 1, j)
    pa = order[starts[f] + i]
    pb = order[starts[f] + j]
    ua = rng.integers(0, ds.n, size=n_pairs - n_in)
    ub = rng.integers(0, ds.n - 1, size=n_pairs - n_in)
    ub = np.where(ub >= ua, ub + 1, ub)
    pairs = np.stack([np.concatenate([pa, ua]), np.concatenate([pb, ub])], axis=1).astype(np.int32)
    pairs = pairs[rng.permutation(len(pairs))]
    ds.pairs = pairs
    ds.meta["workload"] = f"screen-train-{n_pairs}"
    return ds


def clustermerge_large(seed: int = 505) -> Dataset:
    """300,000 proteins in 25,000 Zipf families, lognormal(350, 0.6) clipped to [30, 5000]."""
    return clustermerge_families(300000, 25000, seed, hi=5000)


def max_length_set(L: int = 65535, seed: int = 113) -> Dataset:
    """Proteins at the longest accepted length L: a query (a mutated copy of a
    random ancestor, padded with random residues to L) against eight subjects
    of 0.9 L to L residues sharing it (one item of eight pairs with one query):
    an identical copy, mutated relatives and unrelated proteins; plus a 4,000-
    residue stretch of the query, short proteins and one residue.  Pairs: the
    eight query-subject pairs, some reversed, and the short ones both ways."""
    rng = np.random.default_rng(seed)
    anc = rng.integers(0, N_RES, size=L).astype(np.uint8)
    q = np.concatenate([mutate(rng, anc), rng.integers(0, N_RES, size=L).astype(np.uint8)])[:L]
    seqs = [q]
    for k, n in enumerate((L, L - 1, int(0.98 * L), int(0.96 * L), int(0.94 * L), int(0.93 * L), int(0.92 * L),
                           int(0.9 * L))):
        if k == 0:
            t = q.copy()
        elif k % 2 == 0:
            t = mutate(rng, anc)
        else:
            t = rng.integers(0, N_RES, size=n).astype(np.uint8)
        seqs.append(np.concatenate([t, rng.integers(0, N_RES, size=L).astype(np.uint8)])[:n])
    seqs.append(q[20000:24000].copy())                                  # 9: a stretch of the query
    seqs += [rng.integers(0, N_RES, size=n).astype(np.uint8) for n in (3000, 300, 1)]   # 10, 11, 12
    ds = _pack(seqs, np.full(len(seqs), -1), make_matrix(), dict(seed=seed, workload=f"max-length-{L}"))
    ds.pairs = np.array([(0, k) for k in range(1, 9)] + [(3, 0), (4, 0), (9, 0), (0, 9), (0, 10), (10, 0),
                                                         (11, 0), (0, 12), (12, 3)], np.int32)
    return ds


def random_pairs(rng, n_seqs: int, n_pairs: int) -> np.ndarray:
    a = rng.integers(0, n_seqs, size=n_pairs)
    b = rng.integers(0, n_seqs, size=n_pairs)
    return np.stack([a, b], axis=1).astype(np.int32)


def uniform_pool(n: int, lo: int, hi: int, seed: int) -> Dataset:
    """I.i.d. random sequences with lengths uniform on [lo, hi] (test inputs)."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(lo, hi + 1, size=n)
    seqs = [random_residues(rng, int(L)) for L in lens]
    return _pack(seqs, np.full(n, -1), make_matrix(), dict(seed=seed))


def from_list(seqs, matrix=None) -> Dataset:
    seqs = [np.asarray(s, dtype=np.uint8) for s in seqs]
    return _pack(seqs, np.full(len(seqs), -1), make_matrix() if matrix is None else matrix, {})
