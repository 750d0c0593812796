"""The seeded synthetic workloads follow the recipe they are documented with
(CPU only): family sizes, length distributions, clipping, the throughput pool's
length mix, valid pair lists, and determinism under the seed."""
import numpy as np

import cmgen


def test_clustermerge_20k_recipe():
    """20,000 proteins in 2,000 rank-size Zipf(1.2) families; lengths drawn per
    family from lognormal(median 350, sigma 0.6), clipped to [30, 2,000].  With
    2,000 families the sample median of the per-family lengths has a standard
    error of about 2% and the log standard deviation about 1.6%, so 5% bounds
    leave room for the members' indels."""
    ds = cmgen.clustermerge_families()
    assert ds.n == 20000
    L = np.diff(ds.offsets)
    assert L.min() >= 30 and L.max() <= 2000
    assert ds.residues.max() < 20
    sizes = np.bincount(ds.family)
    assert len(sizes) == 2000 and sizes.sum() == 20000 and sizes.min() >= 1
    assert (np.diff(sizes) <= 0).all()                         # family k is the k-th largest
    assert abs(sizes[0] / sizes[9] / 10 ** 1.2 - 1) < 0.02     # rank-size ratio of ranks 1 and 10
    assert np.array_equal(sizes, cmgen.zipf_sizes(20000, 2000))
    med = np.array([np.median(L[ds.family == f]) for f in range(2000)])
    assert abs(np.median(med) / 350 - 1) < 0.05
    assert abs(np.std(np.log(med)) / 0.6 - 1) < 0.05


def test_zipf_sizes_rounding():
    for n, f in ((20000, 2000), (300000, 25000), (500, 50), (10, 10)):
        z = cmgen.zipf_sizes(n, f)
        assert z.sum() == n and z.min() >= 1 and (np.diff(z) <= 0).all()


def test_throughput_pool_recipe():
    """200,000 proteins, 20% uniform on [1,000, 5,000] and 80% lognormal(300,
    0.6); the lognormal part passes 1,000 with probability about 2.3%, so about
    21.8% of the pool is at least 1,000 long.  1,000,000 pairs of distinct proteins."""
    tp = cmgen.throughput_pool()
    L = np.diff(tp.offsets)
    assert tp.n == 200000 and L.min() >= 30 and L.max() <= 5000
    frac_long = (L >= 1000).mean()
    assert 0.21 < frac_long < 0.226
    short = L[L < 1000]
    assert abs(np.median(short) / 300 - 1) < 0.05
    p = tp.pairs
    assert p.shape == (1000000, 2) and p.min() >= 0 and p.max() < tp.n
    assert (p[:, 0] != p[:, 1]).all()


def test_generators_are_seeded():
    a = cmgen.clustermerge_families(n_seqs=500, n_families=50)
    b = cmgen.clustermerge_families(n_seqs=500, n_families=50)
    assert np.array_equal(a.residues, b.residues) and np.array_equal(a.offsets, b.offsets)
    c = cmgen.clustermerge_families(n_seqs=500, n_families=50, seed=203)
    assert not np.array_equal(a.offsets, c.offsets)
