"""Canonical digests of alignment and clustering outputs (test helpers).

A digest is the SHA-256 of a canonical little-endian int32 array, so that two
results can be compared exactly without storing them:
  * scores / cells: the int32 array as it is, per pair row;
  * clusters: for each cluster in final-set order, [rep, number of members,
    members in cluster order];
  * similar pairs: rows (x, y, score) sorted by (x, y).
"""
import hashlib

import numpy as np


def sha256_i32(a) -> str:
    a = np.ascontiguousarray(np.asarray(a, dtype="<i4"))
    return hashlib.sha256(a.tobytes()).hexdigest()


def clusters_array(clusters) -> np.ndarray:
    """clusters: iterable of (rep, members)."""
    parts = []
    for rep, members in clusters:
        m = np.asarray(members, dtype=np.int64)
        parts.append(np.concatenate([[int(rep), len(m)], m]))
    return np.concatenate(parts).astype(np.int32) if parts else np.zeros(0, np.int32)


def pairs_array(x, y, s) -> np.ndarray:
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    s = np.asarray(s, dtype=np.int64)
    order = np.lexsort((y, x))
    return np.stack([x[order], y[order], s[order]], axis=1).astype(np.int32)


def block_hashes(a, n_blocks: int = 10) -> list:
    """SHA-256 of each of n_blocks equal row ranges (localises a mismatch)."""
    a = np.asarray(a)
    edges = np.linspace(0, len(a), n_blocks + 1).astype(np.int64)
    return [sha256_i32(a[edges[k]:edges[k + 1]]) for k in range(n_blocks)]
