"""Substitution-matrix calibration gate; writes tests/golden/matrix_gate.txt.

Only the RANGES of the matrix are fixed by the workload (diagonal 4..11,
off-diagonal -4..3).  A uniform draw makes unrelated proteins score above the
similarity threshold, so the generator draws off-diagonal values from a skewed
pmf and this gate picks the seed: starting at 1908, the first seed whose matrix
has expected background score E_q[M] <= -1.8 AND whose 99.9th percentile of
oracle scores over 1,000 unrelated pairs of length 2,000 is below 100.
Run: python tests/golden/matrix_gate.py   (calls the CPU oracle only)
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import cmgen  # noqa: E402
from oracle import sw_batch  # noqa: E402

L, N_PAIRS, POOL_SEED = 2000, 1000, 91


def _scores(args):
    seed, k = args
    M = cmgen.make_matrix(seed)
    ds = cmgen.uniform_pool(2 * N_PAIRS, L, L, seed=POOL_SEED)
    pr = np.stack([np.arange(2 * k, 2 * N_PAIRS, 16), np.arange(2 * k + 1, 2 * N_PAIRS, 16)], 1)
    return sw_batch(ds.residues, ds.offsets, pr.astype(np.int32), M, with_end=False)


def main():
    lines = []
    with Pool(8) as pool:
        for seed in range(1908, 2008):
            M = cmgen.make_matrix(seed)
            E = float(M.mean())
            if E > -1.8:
                lines.append(f"seed {seed}: E={E:.4f} fails E<=-1.8")
                continue
            sc = np.concatenate(pool.map(_scores, [(seed, k) for k in range(8)]))
            p999 = float(np.percentile(sc, 99.9))
            ok = p999 < 100
            lines.append(f"seed {seed}: E={E:.4f} unrelated L={L} n={len(sc)} "
                         f"median={np.median(sc):.0f} p99.9={p999:.1f} max={sc.max()} "
                         + ("PASS" if ok else "fails p99.9<100"))
            if ok:
                break
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "matrix_gate.txt")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
