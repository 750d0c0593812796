"""Training of the learned pair screen on the GPU.

Labels come from the GPU Smith-Waterman itself (score >= T); every forward,
backward and Adam step runs in the library's kernels.  This module only
orchestrates: batching, shuffling, held-out threshold calibration.
"""
from __future__ import annotations

import time

import numpy as np

from . import Screen, clustermerge_run, context, kmer_features, sw_score_batch, sync


def label_pairs(residues, offsets, pairs: np.ndarray, matrix, T: int = 120, gap_open: int = -11,
                gap_extend: int = -1, chunk: int = 1 << 21) -> np.ndarray:
    """uint8 labels (score >= T) of host pair rows, scored by the GPU kernels."""
    import torch
    out = np.zeros(len(pairs), np.uint8)
    for k in range(0, len(pairs), chunk):
        p = torch.from_numpy(np.ascontiguousarray(pairs[k:k + chunk], dtype=np.int32)).cuda()
        s = sw_score_batch(residues, offsets, p, matrix, gap_open, gap_extend)
        out[k:k + chunk] = (s >= T).cpu().numpy()
    sync()
    return out


def screen_logits(scr: Screen, feat, pairs: np.ndarray, chunk: int = 1 << 21) -> np.ndarray:
    import torch
    out = np.zeros(len(pairs), np.float32)
    for k in range(0, len(pairs), chunk):
        p = torch.from_numpy(np.ascontiguousarray(pairs[k:k + chunk], dtype=np.int32)).cuda()
        out[k:k + chunk] = scr.infer(feat, p).cpu().numpy()
    return out


def train(scr: Screen, feat, pairs: np.ndarray, labels: np.ndarray, epochs: int = 5, batch: int = 4096,
          lr: float = 1e-3, seed: int = 0, log=None) -> list:
    """Mini-batch Adam over shuffled pairs, the whole run in one library call
    (cm_screen_train); returns the mean loss of each epoch."""
    import torch
    tp = torch.from_numpy(np.ascontiguousarray(pairs, dtype=np.int32)).cuda()
    ty = torch.from_numpy(np.ascontiguousarray(labels, dtype=np.uint8)).cuda()
    steps = scr.train(feat, tp, ty, epochs=epochs, batch=batch, lr=lr, shuffle=True, seed=seed, drop_last=True)
    per = len(steps) // epochs
    hist = [float(steps[e * per:(e + 1) * per].mean()) for e in range(epochs)]
    if log:
        for ep, v in enumerate(hist):
            log(f"screen epoch {ep}: loss {v:.4f}")
    return hist


def calibrate_tau(z: np.ndarray, y: np.ndarray, keep_recall: float = 0.999) -> float:
    """Largest threshold that keeps at least keep_recall of the positives."""
    pos = np.sort(z[y == 1])
    if len(pos) == 0:
        return float(np.min(z)) - 1.0
    k = int(np.floor((1.0 - keep_recall) * len(pos)))
    return float(pos[k]) - 1e-6


def auc(z: np.ndarray, y: np.ndarray) -> float:
    """Area under the ROC curve (rank statistic)."""
    order = np.argsort(z, kind="stable")
    ranks = np.empty(len(z), np.float64)
    ranks[order] = np.arange(1, len(z) + 1)
    npos = int(y.sum())
    nneg = len(y) - npos
    if npos == 0 or nneg == 0:
        return float("nan")
    return float((ranks[y == 1].sum() - npos * (npos + 1) / 2) / (npos * nneg))


def train_on_dataset(ds, n_holdout_frac: float = 0.05, epochs: int = 5, batch: int = 4096, lr: float = 1e-3,
                     seed: int = 1, keep_recall: float = 0.999, log=None) -> tuple:
    """Features, GPU labels, training and calibration on a dataset with ds.pairs.

    Returns (screen, tau, info dict).
    """
    import torch
    t0 = time.perf_counter()
    res = torch.from_numpy(ds.residues).cuda()
    off = torch.from_numpy(ds.offsets).cuda()
    feat = kmer_features(res, off)
    labels = label_pairs(res, off, ds.pairs, ds.matrix)
    t1 = time.perf_counter()
    n_hold = int(len(ds.pairs) * n_holdout_frac)
    tr_p, tr_y = ds.pairs[n_hold:], labels[n_hold:]
    ho_p, ho_y = ds.pairs[:n_hold], labels[:n_hold]
    scr = Screen(seed, context())
    hist = train(scr, feat, tr_p, tr_y, epochs, batch, lr, seed, log)
    sync()
    t2 = time.perf_counter()
    z = screen_logits(scr, feat, ho_p)
    tau = calibrate_tau(z, ho_y, keep_recall)
    info = dict(n_train=int(len(tr_p)), n_holdout=int(n_hold), positive_frac=float(labels.mean()),
                loss_per_epoch=hist, holdout_auc=auc(z, ho_y), tau=tau,
                holdout_pos_kept=float((z[ho_y == 1] >= tau).mean()) if ho_y.sum() else float("nan"),
                holdout_neg_dropped=float((z[ho_y == 0] < tau).mean()) if (ho_y == 0).sum() else float("nan"),
                label_s=t1 - t0, train_s=t2 - t1)
    return scr, tau, info


def calibrate_on_clustermerge(scr: Screen, ds, keep_recall: float = 0.999, T: int = 120) -> tuple:
    """Threshold from the candidates the screen will judge: a plain
    ClusterMerge run on a separate family set records every pair it scores in
    the merge stage (representative and exchange alignments); tau keeps
    keep_recall of those scoring >= T.  Returns (tau, info)."""
    import torch
    t0 = time.perf_counter()
    res = torch.from_numpy(ds.residues).cuda()
    off = torch.from_numpy(ds.offsets).cuda()
    feat = kmer_features(res, off)
    g = clustermerge_run(res, off, ds.matrix, T=T, record_candidates=True, max_result_pairs=0)
    pairs, scores = g["candidates"], g["candidate_scores"]
    z = screen_logits(scr, feat, pairs)
    y = (scores >= T).astype(np.uint8)
    tau = calibrate_tau(z, y, keep_recall)
    info = dict(workload=f"plain ClusterMerge candidates of a separate {ds.n}-protein family set "
                         f"(seed {ds.meta.get('seed')})", n_candidates=int(len(pairs)),
                positive_frac=float(y.mean()), tau=tau,
                candidate_pos_kept=float((z[y == 1] >= tau).mean()) if y.sum() else float("nan"),
                candidate_neg_dropped=float((z[y == 0] < tau).mean()) if (y == 0).sum() else float("nan"),
                auc=auc(z, y), seconds=time.perf_counter() - t0)
    return tau, info
