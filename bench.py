#!/usr/bin/env python3
"""Benchmark of the ClusterMerge hot path on one MI355X.

Step = one ClusterMerge run (Algorithm 2 over Algorithm 1, the protein
transitivity test of Section 4 and the final in-cluster all-against-all of
Section 6.1) over 20,000 synthetic proteins in 2,000 Zipf(1.2) families
(lognormal lengths, median 350, sigma 0.6, clipped to 30-2,000), with the
sequence store already resident in HBM.  Every alignment is Smith-Waterman
(Gotoh, gap open -11, extend -1, seeded 20x20 matrix), int32, bit-exact.

Printed (rank 0, one JSON line): whole-step throughput in GCUPS (aligned
cells / wall time of the step), the score kernel's achieved op rate against
its VALU roofline (HIP events around every launch in the timed region; the
packed 16-bit kernel against the packed 16-bit peak, and the same cell rate
against the int32 formulation's peak), ClusterMerge time and pair recall
(found / all-vs-all truth count), a throughput leg on 1,000,000 random pairs
of a 200,000-protein pool, and the CPU oracle's rate on a bounded sample of
the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SW GCUPS (bit-exact int32); ClusterMerge time + pair recall, learned vs plain"
OPS_PER_CELL = 8                       # int32: add, max3, max, add, add, max3, add, max3
PEAK_INT32_OPS = 256 * 64 * 2.4e9      # CUs x lanes/clk x clock (MI355X)
# packed 16-bit kernels (biased values, maxima as binary16 maximum3), per cell:
# saturating add (diagonal + substitution), maximum3 (H), saturating subtract
# (open), subtract + maximum3 (E), subtract + maximum3 (F), half a maximum3
# (best over two rows)
PK_OPS_PER_CELL = 7.5
PEAK_PK16_OPS = 256 * 64 * 2 * 2.4e9   # CUs x lanes/clk x 16-bit halves x clock


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per score pass (k_sw_pkq + k_sw_pk) from the committed
    PMC summary, if it was taken on the current kernel source; else None."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "k_sw_pkq_traffic_clustermerge_20k.txt")
    src = os.path.join(ROOT, "paper_1908_10574_amd", "csrc", "sw_kernels.hip")
    if not os.path.exists(prof):
        return None
    kv = dict(line.split("=", 1) for line in open(prof).read().splitlines() if "=" in line and not line.startswith("#"))
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get("kernel_source_sha256", "").strip() != digest:
        return None
    return float(kv["traffic_bytes_per_launch"])


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


_POOL = {}


def _pool_init(res, off, mat):
    _POOL["res"], _POOL["off"], _POOL["mat"] = res, off, mat


def _pool_score(pairs):
    from oracle import sw_batch
    return sw_batch(_POOL["res"], _POOL["off"], pairs, _POOL["mat"], with_end=False)


def cpu_baseline(ds, n_sample, tp_pairs=48000, workers=0, T=120, mT=166, mU=15):
    """The CPU oracle (scalar C Smith-Waterman + sequential Algorithms 1-2 in
    Python), run before anything touches the GPU:
      * value: the ClusterMerge oracle on the first n_sample proteins of the
        same store, one thread;
      * single_core_allvsall_100: the oracle's Smith-Waterman on the 4,950
        pairs of the 100-protein all-against-all set, one thread;
      * all_cores_throughput_sample: the first tp_pairs pairs of the
        1,000,000-pair throughput batch scored by independent oracle
        processes (one per host core, up to 16), contiguous chunks."""
    import multiprocessing as mp
    import numpy as np
    import cmgen
    from oracle import clustermerge as ocm
    from oracle import sw_batch
    nproc = os.cpu_count() or 1
    workers = workers or min(16, nproc)
    off = ds.offsets[: n_sample + 1]
    res = ds.residues[: int(off[-1])]
    judge = ocm.ProteinJudge(res, off, ds.matrix, T, mT, mU)
    t0 = time.perf_counter()
    clusters, _ = ocm.bottom_up_merge(n_sample, judge)
    ocm.similar_pairs(clusters, judge.score, T)
    dt = time.perf_counter() - t0
    L = np.diff(off).astype(np.float64)
    cells = sum(L[x] * L[y] for x, y in judge._score)
    out = dict(value=cells / dt / 1e9, unit="GCUPS", cores=1, kind="oracle",
               sample=f"ClusterMerge oracle on the first {n_sample} proteins of the same store "
                      f"({len(judge._score)} alignments, {cells:.3e} cells, {dt:.1f} s, single thread)",
               nproc=nproc, cpu_model=cpu_model(), compiler="gcc -O2 -std=c99 (scalar C Smith-Waterman)")
    small = cmgen.allvsall_small()
    Ls = small.lengths().astype(np.float64)
    c1 = float((Ls[small.pairs[:, 0]] * Ls[small.pairs[:, 1]]).sum())
    t0 = time.perf_counter()
    sw_batch(small.residues, small.offsets, small.pairs, small.matrix, with_end=False)
    d1 = time.perf_counter() - t0
    out["single_core_allvsall_100"] = dict(pairs=int(len(small.pairs)), cells=c1, seconds=d1, gcups=c1 / d1 / 1e9)
    tp = cmgen.throughput_pool()
    pr = tp.pairs[:tp_pairs]
    Lt = tp.lengths().astype(np.float64)
    c2 = float((Lt[pr[:, 0]] * Lt[pr[:, 1]]).sum())
    chunks = np.array_split(pr, workers * 4)
    with mp.get_context("fork").Pool(workers, initializer=_pool_init,
                                      initargs=(tp.residues, tp.offsets, tp.matrix)) as pool:
        t0 = time.perf_counter()
        pool.map(_pool_score, chunks, chunksize=1)
        d2 = time.perf_counter() - t0
    out["all_cores_throughput_sample"] = dict(pairs=int(len(pr)), cells=c2, processes=workers, seconds=d2,
                                              gcups=c2 / d2 / 1e9)
    return out


def sampled_recall(cm, res, off, M, clusters, n, k_sample, seed=7, T=120, chunk=1 << 23):
    """Pair recall estimated from k_sample elements x drawn uniformly: every
    (x, y), y != x, is scored on the GPU; truth(x) = {y : score >= T};
    found(x) = truth(x) restricted to the y sharing a final cluster with x.
    Ratio estimate sum(found) / sum(truth) with a percentile bootstrap interval."""
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    xs = np.sort(rng.choice(n, size=k_sample, replace=False)).astype(np.int32)
    sampled = np.zeros(n, bool)
    sampled[xs] = True
    together = {int(x): [] for x in xs}
    for _, members in clusters:
        m = np.asarray(members)
        for x in m[sampled[m]]:
            together[int(x)].append(m)
    ys = np.arange(n, dtype=np.int32)
    truth = np.zeros(k_sample, np.int64)
    found = np.zeros(k_sample, np.int64)
    cells = 0.0
    L = np.diff(np.asarray(off.cpu()) if hasattr(off, "cpu") else off).astype(np.float64)
    t0 = time.perf_counter()
    per = max(1, chunk // n)
    for b in range(0, k_sample, per):
        xb = xs[b:b + per]
        pr = np.stack([np.repeat(xb, n), np.tile(ys, len(xb))], 1).astype(np.int32)
        pr = pr[pr[:, 0] != pr[:, 1]]
        cells += float((L[pr[:, 0]] * L[pr[:, 1]]).sum())
        sc = cm.sw_score_batch(res, off, torch.from_numpy(pr).cuda(), M).cpu().numpy()
        for i, x in enumerate(xb):
            sel = pr[:, 0] == x
            yt = pr[sel, 1][sc[sel] >= T]
            mem = np.unique(np.concatenate(together[int(x)])) if together[int(x)] else np.zeros(0, np.int32)
            truth[b + i] = len(yt)
            found[b + i] = int(np.isin(yt, mem).sum())
    dt = time.perf_counter() - t0
    est = found.sum() / max(truth.sum(), 1)
    boot = []
    for _ in range(2000):
        idx = rng.integers(0, k_sample, size=k_sample)
        boot.append(found[idx].sum() / max(truth[idx].sum(), 1))
    lo, hi = np.percentile(boot, [2.5, 97.5])
    return dict(recall=float(est), ci95=[float(lo), float(hi)], sampled_elements=int(k_sample),
                sampled_truth_pairs=int(truth.sum()), sampled_found_pairs=int(found.sum()),
                sample_s=dt, sample_gcups=cells / dt / 1e9)


def truth_pairs(cm, res, off, M, n, T_min, chunk=1 << 24):
    """Every (x, y), x < y, of the store scoring at least T_min, with its
    score: the all-vs-all triangle scored on the GPU in row blocks of about
    `chunk` pairs (pair lists built on the host)."""
    import numpy as np
    import torch
    xs, ys, ss = [], [], []
    x0 = 0
    while x0 < n - 1:
        x1 = x0
        tot = 0
        while x1 < n - 1 and tot + (n - 1 - x1) <= max(chunk, n):
            tot += n - 1 - x1
            x1 += 1
        cnt = n - 1 - np.arange(x0, x1)
        x = np.repeat(np.arange(x0, x1, dtype=np.int64), cnt)
        start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
        y = np.arange(tot, dtype=np.int64) - np.repeat(start, cnt) + x + 1
        pr = torch.from_numpy(np.stack([x, y], 1).astype(np.int32)).cuda()
        sc = cm.sw_score_batch(res, off, pr, M)
        keep = sc >= T_min
        xs.append(pr[keep, 0].cpu().numpy())
        ys.append(pr[keep, 1].cpu().numpy())
        ss.append(sc[keep].cpu().numpy())
        x0 = x1
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ss)


def traceback_rate(cm, ds, res, off, found, n_gpu=200000, n_cpu=300, seed=11):
    """Alignment columns of found pairs: GPU rate on a sample of n_gpu pairs
    (score + end, start, columns timed separately) and the oracle's rate on
    n_cpu of them; rates in box cells per second."""
    import numpy as np
    import torch
    from oracle import traceback_batch
    rng = np.random.default_rng(seed)
    pick = found[rng.choice(len(found), size=min(n_gpu, len(found)), replace=False)]
    pr = torch.from_numpy(np.ascontiguousarray(pick, dtype=np.int32)).cuda()
    M = ds.matrix
    times = {}
    torch.cuda.synchronize()
    t = time.perf_counter()
    sc, ea, eb = cm.sw_score_batch(res, off, pr, M, return_end=True)
    torch.cuda.synchronize()
    times["score_end_s"] = time.perf_counter() - t
    t = time.perf_counter()
    sa, sb = cm.sw_span_batch(res, off, pr, M, sc, ea, eb, 0)
    torch.cuda.synchronize()
    times["span_s"] = time.perf_counter() - t
    t = time.perf_counter()
    ops, op_off, n_ops = cm.sw_traceback_batch(res, off, pr, M, sc, ea, eb, sa, sb)
    torch.cuda.synchronize()
    times["traceback_s"] = time.perf_counter() - t
    cm.sync()
    box = ((ea - sa + 1).double() * (eb - sb + 1).double() * (sc > 0).double()).sum().item()
    cols = int(n_ops.clamp(min=0).sum().item())
    sub = pick[:n_cpu]
    t = time.perf_counter()
    want, _ = traceback_batch(ds.residues, ds.offsets, sub, M)
    t_cpu = time.perf_counter() - t
    spans = torch.stack([sc, ea, eb, sa, sb], 1)[:n_cpu].cpu().numpy().astype(np.float64)
    cpu_box = float(((spans[:, 1] - spans[:, 3] + 1) * (spans[:, 2] - spans[:, 4] + 1) * (spans[:, 0] > 0)).sum())
    got = cm.columns_as_strings(ops[: int(op_off[n_cpu].item()) or 1], op_off[: n_cpu + 1], n_ops[:n_cpu])
    out = dict(pairs=int(len(pick)), box_cells=box, columns=cols, gpu_box_cells_per_s=box / times["traceback_s"],
               cpu_baseline=dict(value=cpu_box / t_cpu, unit="box cells/s", cores=1, kind="oracle",
                                 sample=f"the first {len(sub)} sampled pairs, C oracle traceback"),
               agrees_with_oracle_on_sample=bool(got == want), **times)
    log(f"traceback: {len(pick)} found pairs, {box:.3g} box cells in {times['traceback_s']:.3f} s "
        f"({out['gpu_box_cells_per_s'] / 1e9:.1f} G cells/s); oracle {cpu_box / t_cpu / 1e6:.1f} M cells/s")
    return out


def cluster_profile(clusters):
    import numpy as np
    sz = np.array([len(m) for _, m in clusters], np.int64)
    return dict(n_clusters=int(len(sz)), largest=int(sz.max()) if len(sz) else 0,
                frac_1_to_4=float((sz <= 4).mean()), frac_over_10=float((sz > 10).mean()),
                frac_over_100=float((sz > 100).mean()), frac_over_1000=float((sz > 1000).mean()))


def parameter_sweep(cm, ds, res, off, n_seqs, n_families):
    """Sensitivity to T, mT and mU (missed similar pairs and their scores,
    clusters, comparisons, time) and to family divergence (substitution rate
    of the members), on the ClusterMerge workload."""
    import numpy as np
    import torch
    import cmgen
    M = ds.matrix
    n = ds.n
    all_pairs = n * (n - 1) // 2
    g = cm.clustermerge_run(res, off, M)                          # warm
    traceback = traceback_rate(cm, ds, res, off, g["pairs"])
    t0 = time.perf_counter()
    tx, ty, ts = truth_pairs(cm, res, off, M, n, 100)
    t_truth = time.perf_counter() - t0
    tkey = tx.astype(np.int64) * n + ty
    marks = [150, 200, 300, 500, 1000]

    def one(T, mT, mU):
        t = time.perf_counter()
        g = cm.clustermerge_run(res, off, M, T=T, mT=mT, mU=mU)
        dt = time.perf_counter() - t
        st = g["stats"]
        sel = ts >= T
        truth_keys, truth_sc = tkey[sel], ts[sel]
        fp = np.asarray(g["pairs"], np.int64)
        fkey = np.sort(fp[:, 0] * n + fp[:, 1]) if len(fp) else np.zeros(0, np.int64)
        pos = np.clip(np.searchsorted(fkey, truth_keys), 0, max(len(fkey) - 1, 0))
        hit = (fkey[pos] == truth_keys) if len(fkey) else np.zeros(len(truth_keys), bool)
        miss = truth_sc[~hit]
        compared = st["rep_comparisons"] + st["exchange_alignments"] + st["final_candidates"]
        row = dict(T=T, mT=mT, mU=mU, time_s=dt, truth_pairs=int(len(truth_keys)), found_pairs=int(hit.sum()),
                   recall=float(hit.mean()) if len(hit) else 1.0, missed_pairs=int(len(miss)),
                   missed_median_score=float(np.median(miss)) if len(miss) else None,
                   missed_mean_score=float(miss.mean()) if len(miss) else None,
                   missed_max_score=int(miss.max()) if len(miss) else None,
                   missed_at_least={str(m): int((miss >= m).sum()) for m in marks},
                   comparisons=int(compared), comparisons_vs_all_pairs=compared / all_pairs,
                   aligned_pairs=int(st["aligned_pairs"]), full_merges=int(st["full_merges"]),
                   exchanges=int(st["exchanges"]))
        row.update(cluster_profile(g["clusters"]))
        log(f"sweep T={T} mT={mT} mU={mU}: {dt:.2f} s, recall {row['recall']:.6f}, "
            f"{row['missed_pairs']} missed (median score {row['missed_median_score']}), {row['n_clusters']} clusters")
        return row

    # incremental classification: the last 5% of the proteins against a
    # clustering of the first 95%
    n_prev = n - n // 20
    prev = cm.clustermerge_run(res, off[: n_prev + 1].contiguous(), M)
    t = time.perf_counter()
    ext = cm.clustermerge_extend(res, off, M, prev["clusters"], n_prev, prev["pairs"], prev["scores"])
    t_ext = time.perf_counter() - t
    sel = ts >= 120
    fp = np.asarray(ext["pairs"], np.int64)
    fkey = np.sort(fp[:, 0] * n + fp[:, 1])
    hit = np.isin(tkey[sel], fkey, assume_unique=True)
    new_truth = sel & (ty >= n_prev)                 # true pairs involving a new protein
    hit_new = np.isin(tkey[new_truth], fkey, assume_unique=True)
    st = ext["stats"]
    incremental = dict(n_prev=n_prev, n_new=n - n_prev, time_s=t_ext, prev_time_s=prev["stats"]["t_total_s"],
                       recall=float(hit.mean()), recall_pairs_with_new=float(hit_new.mean()),
                       n_clusters=int(st["n_clusters"]), rep_comparisons=int(st["rep_comparisons"]),
                       aligned_pairs=int(st["aligned_pairs"]), cache_hits=int(st["cache_hits"]))
    log(f"incremental: {n - n_prev} proteins against {n_prev} in {t_ext:.2f} s, recall {incremental['recall']:.6f} "
        f"(pairs with a new protein {incremental['recall_pairs_with_new']:.6f})")
    rows = [one(T, mT, 15) for T in (100, 120, 140) for mT in (140, 166, 200, 250)]
    rows += [one(120, 166, mU) for mU in (5, 30, 60)]
    comp = []
    for sub in (0.20, 0.30, 0.40):
        d2 = cmgen.clustermerge_families(n_seqs=n_seqs, n_families=n_families, sub_rate=sub)
        r2 = torch.from_numpy(d2.residues).cuda()
        o2 = torch.from_numpy(d2.offsets).cuda()
        cm.clustermerge_run(r2, o2, d2.matrix, max_result_pairs=0)       # warm
        t = time.perf_counter()
        g = cm.clustermerge_run(r2, o2, d2.matrix, max_result_pairs=0)
        dt = time.perf_counter() - t
        truth, _ = cm.allvsall_count(r2, o2, d2.matrix)
        st = g["stats"]
        compared = st["rep_comparisons"] + st["exchange_alignments"] + st["final_candidates"]
        row = dict(sub_rate=sub, time_s=dt, recall=st["n_similar_pairs"] / max(truth, 1),
                   truth_pairs=int(truth), comparisons_vs_all_pairs=compared / all_pairs,
                   rep_comparisons=int(st["rep_comparisons"]), full_merges=int(st["full_merges"]),
                   exchanges=int(st["exchanges"]), aligned_cells=float(st["aligned_cells"]))
        row.update(cluster_profile(g["clusters"]))
        log(f"composition sub_rate={sub}: {dt:.2f} s, {row['n_clusters']} clusters, recall {row['recall']:.6f}")
        comp.append(row)
    return dict(workload=ds.meta.get("workload"), truth_scoring_s=t_truth, all_pairs=all_pairs,
                incremental=incremental, traceback=traceback, parameters=rows, composition=comp)


def throughput_leg(cm, ctx, args, out, log):
    """The 1,000,000-pair throughput batch: optional autotuning of the score
    pass over the batch (its table goes to out["autotune"]), then one warm
    batch and three timed batches (HIP events around the batches and around
    every score-kernel launch)."""
    import numpy as np
    import torch
    import cmgen
    dev = torch.device("cuda:0")
    tp = cmgen.throughput_pool(n_pairs=args.throughput_pairs)
    M = tp.matrix
    r2 = torch.from_numpy(tp.residues).to(dev)
    o2 = torch.from_numpy(tp.offsets).to(dev)
    p2 = torch.from_numpy(tp.pairs).to(dev)
    L = tp.lengths().astype(np.float64)
    tcells = float((L[tp.pairs[:, 0]] * L[tp.pairs[:, 1]]).sum())
    plan0 = ctx.get_plan(0)
    if args.autotune_pairs > 0:
        # the autotuner picks the score pass's plan on a sample of the batch
        # (every candidate must agree on every output); the leg runs with it
        t = time.perf_counter()
        table = ctx.autotune(r2, o2, p2[:args.autotune_pairs], M, 0)
        tune_s = time.perf_counter() - t
        chosen = ctx.get_plan(0)
        out["autotune"] = dict(sample_pairs=args.autotune_pairs, seconds=tune_s,
                               table=[dict(kernel=k, rmax=r, blocks_per_cu=b, ms=ms) for k, r, b, ms in table],
                               chosen=dict(kernel=chosen[0], rmax=chosen[1], blocks_per_cu=chosen[2]),
                               default=dict(kernel=plan0[0], rmax=plan0[1], blocks_per_cu=plan0[2]))
        log(f"autotune on {args.autotune_pairs} pairs: {len(table)} plans in {tune_s:.2f} s, chosen {chosen[:3]}")
    tp_packed = ctx.get_plan(0)[0] >= 1
    tp_opc, tp_peak = (PK_OPS_PER_CELL, PEAK_PK16_OPS) if tp_packed else (OPS_PER_CELL, PEAK_INT32_OPS)
    cm.sw_score_batch(r2, o2, p2, M)
    ctx.sync()
    ctx.set_timing(True)
    n0, s0 = ctx.kernel_time(0)
    cc0 = ctx.cells_computed(0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 3
    for _ in range(reps):
        cm.sw_score_batch(r2, o2, p2, M)
    e1.record()
    ctx.sync()
    n1, s1 = ctx.kernel_time(0)
    computed = (ctx.cells_computed(0) - cc0) / reps
    ctx.set_timing(False)
    bt = e0.elapsed_time(e1) / 1e3 / reps
    ks = (s1 - s0) / max(n1 - n0, 1)
    res = dict(
        workload=f"throughput-{args.throughput_pairs}: random pairs of a 200,000-protein pool, 80% "
                 "lognormal(300, 0.6) / 20% U[1000,5000]", cells=tcells, batch_s=bt, gcups=tcells / bt / 1e9,
        plan=list(ctx.get_plan(0)[:3]),
        kernel_s=ks, kernel_gcups=tcells / ks / 1e9, kernel_roofline_frac=tp_opc * tcells / ks / tp_peak,
        kernel_frac_8ops_packed_peak=8 * tcells / ks / PEAK_PK16_OPS,
        int32_formulation_frac=OPS_PER_CELL * tcells / ks / PEAK_INT32_OPS,
        # cells the kernels computed (strip ramps, padded rows, columns past a
        # shorter pair's end) per cell the pairs have
        computed_cells=computed, computed_per_counted_cell=computed / tcells,
        kernel_frac_8ops_on_computed_cells=8 * computed / ks / PEAK_PK16_OPS)
    log(f"throughput: {tcells / bt / 1e9:.1f} GCUPS batch, kernel {tcells / ks / 1e9:.1f} GCUPS, "
        f"{computed / tcells:.3f} computed cells per counted cell")
    if args.autotune_pairs > 0:
        ctx.set_plan(0, *plan0[:3])     # the ClusterMerge legs keep the default plan
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["clustermerge-20k", "clustermerge-300k"], default="clustermerge-20k",
                    help="clustermerge-300k: 300,000 proteins, 25,000 families, lengths clipped to 30-5,000; "
                         "recall from a sample of elements (use --steps 1 --warmup 0)")
    ap.add_argument("--recall-sample", type=int, default=256,
                    help="clustermerge-300k: elements whose pairs with every protein define the recall sample")
    ap.add_argument("--sub-rate", type=float, default=0.30,
                    help="member substitution rate of the family generator (dataset composition; 0.30 = the workload)")
    ap.add_argument("--n-seqs", type=int, default=20000)
    ap.add_argument("--n-families", type=int, default=2000)
    ap.add_argument("--throughput-pairs", type=int, default=1000000)
    ap.add_argument("--cpu-sample", type=int, default=250)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--no-throughput", action="store_true")
    ap.add_argument("--no-screen", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark: T / mT / mU and family-divergence sweep (one JSON line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 256 MiB device copy first (reference for HBM byte counters)")
    ap.add_argument("--screen-pairs", type=int, default=2000000)
    ap.add_argument("--screen-epochs", type=int, default=5)
    ap.add_argument("--screen-keep", type=float, default=0.999)
    ap.add_argument("--only-throughput", action="store_true",
                    help="only the 1,000,000-pair throughput leg (for profiling its kernels); prints its JSON")
    ap.add_argument("--graph-steps", type=int, default=3,
                    help="steps timed again with graph-captured waves (0: skip)")
    ap.add_argument("--autotune-pairs", type=int, default=1000000,
                    help="pairs of the throughput batch the autotuner times every plan on (0: skip); a small "
                         "sample favours plans with short tails over plans with high throughput")
    ap.add_argument("--screen-calibration-seed", type=int, default=406,
                    help="family set whose plain-run candidates calibrate the screen threshold (0: the training "
                         "holdout)")
    ap.add_argument("--screen-min-product", type=int, default=64,
                    help="representative pairs of clusters whose sizes multiply to at least this bypass the screen")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; the sharding it "
              "would take is described in the design notes (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import cmgen

    # the CPU oracle runs first, while no GPU state exists (its process pool
    # forks this process)
    cpu = None
    if not args.no_cpu_baseline and not args.sweep:
        base_ds = cmgen.clustermerge_families(n_seqs=args.n_seqs, n_families=args.n_families) \
            if args.workload != "clustermerge-300k" else cmgen.clustermerge_large()
        cpu = cpu_baseline(base_ds, args.cpu_sample)
        del base_ds
        log(f"cpu baseline: {cpu['value']:.3f} GCUPS (one thread), "
            f"{cpu['all_cores_throughput_sample']['gcups']:.2f} GCUPS on "
            f"{cpu['all_cores_throughput_sample']['processes']} processes ({cpu['cpu_model']}, nproc {cpu['nproc']})")

    import torch
    import paper_1908_10574_amd as cm

    dev = torch.device("cuda:0")
    if args.only_throughput:
        extra = {}
        res_tp = throughput_leg(cm, cm.context(), args, extra, log)
        print(json.dumps(dict(sw_throughput=res_tp, **extra)), flush=True)
        return
    large = args.workload == "clustermerge-300k"
    if large:
        args.n_seqs, args.n_families = 300000, 25000
        ds = cmgen.clustermerge_large()
    else:
        ds = cmgen.clustermerge_families(n_seqs=args.n_seqs, n_families=args.n_families, sub_rate=args.sub_rate)
    # the large store reports counts and the set hash only (billions of pairs)
    cm_kw = dict(max_result_pairs=0) if large else {}
    res = torch.from_numpy(ds.residues).to(dev)
    off = torch.from_numpy(ds.offsets).to(dev)
    M = ds.matrix
    ctx = cm.context()
    torch.cuda.synchronize()
    log(f"store: {ds.n} proteins, {len(ds.residues)} residues")

    if args.sweep:
        print(json.dumps(dict(sweep=parameter_sweep(cm, ds, res, off, args.n_seqs, args.n_families))), flush=True)
        return

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for w in range(args.warmup):
        g = cm.clustermerge_run(res, off, M, **cm_kw)
        log(f"warmup {w}: {g['stats']['t_total_s']:.2f} s")
    torch.cuda.synchronize()
    stats = []
    cc0 = ctx.cells_computed(0)
    t0 = time.perf_counter()
    if large:
        os.environ["CM_LOG"] = "1"          # per-level progress lines
    for k in range(args.steps):
        g = cm.clustermerge_run(res, off, M, **cm_kw)
        stats.append(g["stats"])
        log(f"step {k}: {g['stats']['t_total_s']:.2f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    computed = ctx.cells_computed(0) - cc0      # cells the score kernels computed (padding and ramps included)
    step_s = wall / args.steps
    s = stats[-1]
    cells = s["aligned_cells"]
    # headline: the cells the method needs (Algorithm 1's comparisons, its
    # exchanges' tests, the final stage's pairs not already scored) per second
    # of the whole step; executed cells (with speculation) are reported beside
    req_cells = s["required_cells"]
    value = req_cells / step_s / 1e9
    k_launch = sum(x["sw_launches"] for x in stats)
    k_sec = sum(x["sw_kernel_s"] for x in stats)
    k_cells = sum(x["aligned_cells"] for x in stats)
    packed = ctx.get_plan(0)[0] >= 1         # packed 16-bit kernels (two-profile or shared-query)
    opc, peak = (PK_OPS_PER_CELL, PEAK_PK16_OPS) if packed else (OPS_PER_CELL, PEAK_INT32_OPS)
    achieved = opc * k_cells / k_sec
    roofline = dict(bound="alu", achieved=achieved / 1e12, peak=peak / 1e12,
                    unit="TOP/s (16-bit packed)" if packed else "TOP/s (int32)",
                    frac=achieved / peak, traffic=None if large else measured_traffic(),
                    kernel=({1: "k_sw_pk (packed 16-bit Smith-Waterman score kernel; saturated pairs re-run in int32)",
                             2: "k_sw_pkq + k_sw_pk (packed 16-bit Smith-Waterman score kernels: items of eight pairs "
                                "sharing a query, then the rest; saturated pairs re-run in int32)"}
                            .get(ctx.get_plan(0)[0], "k_sw (int32 Smith-Waterman score kernel)")),
                    ops_per_cell=opc, launches=k_launch, avg_launch_ms=1e3 * k_sec / max(k_launch, 1),
                    computed_per_counted_cell=computed / k_cells if k_cells else None,
                    frac_on_computed_cells=opc * computed / k_sec / peak,
                    ops_per_launch=opc * k_cells / max(k_launch, 1),
                    cell_rate_gcups=k_cells / k_sec / 1e9,
                    int32_formulation_frac=OPS_PER_CELL * k_cells / k_sec / PEAK_INT32_OPS)

    probes = {}
    for name, kind in (("i32_add", cm.CM_PROBE_I32_ADD), ("i32_max3", cm.CM_PROBE_I32_MAX3),
                       ("pk16_add", cm.CM_PROBE_PK16_ADD), ("pk16_maximum3", cm.CM_PROBE_PK16_MAX3)):
        ops, clk = cm.probe_valu(kind)
        probes[name] = ops / 1e12
        probes[name + "_clock_ghz"] = clk / 1e9
    roofline["measured_peak"] = dict(unit="TOP/s", **probes)
    mp_peak = probes["pk16_maximum3"] if packed else probes["i32_max3"]
    roofline["frac_of_measured_peak"] = achieved / (mp_peak * 1e12)
    log(f"measured VALU peaks (TOP/s): {probes}")
    out = dict(metric=METRIC, value=value, unit="GCUPS", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=1e3 * step_s, higher_is_better=True, scaling="weak", vs_baseline=None,
               # the score pass computes in packed 16-bit integers (int32 for end and start cells and
               # for pairs that saturate); every output is the exact int32 result
               dtype="i16x2" if packed else "i32", data="synthetic",
               config=dict(workload=f"clustermerge-{ds.n}: {args.n_families} Zipf(1.2) families, lognormal "
                                    f"lengths median 350 sigma 0.6 clipped 30-{5000 if large else 2000}"
                                    + (f", substitution rate {args.sub_rate}" if args.sub_rate != 0.30 else "")
                                    + ", T=120 mT=166 mU=15, gap -11/-1, matrix seed 1917, plain method",
                           n_seqs=ds.n, residues=int(len(ds.residues))),
               roofline=roofline)
    out["clustermerge"] = dict(
        time_s=step_s, required_cells=req_cells, required_gcups=req_cells / step_s / 1e9,
        executed_gcups=cells / step_s / 1e9, speculative_cell_frac=1.0 - req_cells / max(cells, 1.0),
        aligned_cells=cells, aligned_pairs=s["aligned_pairs"], rep_comparisons=s["rep_comparisons"],
        exchange_alignments=s["exchange_alignments"], full_merges=s["full_merges"], exchanges=s["exchanges"],
        n_clusters=s["n_clusters"], n_similar_pairs=s["n_similar_pairs"], waves=s["waves"],
        gpu_s=s["t_gpu_s"], host_s=s["t_host_s"], merge_s=s["t_merge_s"], final_s=s["t_final_s"],
        score_kernel_s=s["sw_kernel_s"], end_kernel_s=s["end_kernel_s"], end_pairs=s["end_pairs"],
        speculative_pairs=s["speculative_pairs"], final_candidates=s["final_candidates"],
        cache_hits=s["cache_hits"], rounds=s["rounds"])

    if not large and args.graph_steps > 0:
        # the same step with every wave replayed as a captured graph
        ctx.set_graphs(True)
        cm.clustermerge_run(res, off, M, **cm_kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.graph_steps):
            gg = cm.clustermerge_run(res, off, M, **cm_kw)
        torch.cuda.synchronize()
        g_step = (time.perf_counter() - t0) / args.graph_steps
        ctx.set_graphs(False)
        out["clustermerge"]["graphs"] = dict(time_s=g_step, steps=args.graph_steps, vs_eager=step_s / g_step,
                                             same_pairs=gg["stats"]["pair_set_hash"] == s["pair_set_hash"])
        log(f"graph-captured waves: {g_step:.3f} s/step against {step_s:.3f} s eager")

    plain_clusters = g["clusters"]
    if not args.no_recall and large:
        out["clustermerge"]["recall_sample"] = sampled_recall(cm, res, off, M, plain_clusters, ds.n,
                                                              args.recall_sample)
        out["clustermerge"]["recall"] = out["clustermerge"]["recall_sample"]["recall"]
        log(f"sampled recall {out['clustermerge']['recall']:.5f}")
    elif not args.no_recall:
        t = time.perf_counter()
        truth, tcells = cm.allvsall_count(res, off, M)
        tt = time.perf_counter() - t
        out["clustermerge"].update(truth_pairs=truth, recall=s["n_similar_pairs"] / max(truth, 1),
                                   allvsall_s=tt, allvsall_gcups=tcells / tt / 1e9)
        log(f"all-vs-all truth {truth} in {tt:.1f} s")

    if not args.no_screen:
        from paper_1908_10574_amd import screen_train
        t = time.perf_counter()
        tr = cmgen.screen_training(seed=404, n_pairs=args.screen_pairs)
        gen_s = time.perf_counter() - t
        scr, tau, info = screen_train.train_on_dataset(tr, epochs=args.screen_epochs, seed=1,
                                                       keep_recall=args.screen_keep, log=log)
        del tr
        calib = None
        if args.screen_calibration_seed > 0:
            # tau from the candidates of a plain run on a third family set
            cal = cmgen.clustermerge_families(n_seqs=min(args.n_seqs, 20000), n_families=min(args.n_families, 2000),
                                              seed=args.screen_calibration_seed, sub_rate=args.sub_rate)
            tau, calib = screen_train.calibrate_on_clustermerge(scr, cal, keep_recall=args.screen_keep)
            del cal
            log(f"tau from {calib['n_candidates']} ClusterMerge candidates: {tau:.3f} (holdout tau {info['tau']:.3f})")
        kw = dict(screen=scr, screen_tau=tau, screen_min_product=args.screen_min_product, **cm_kw)
        if not large:
            g = cm.clustermerge_run(res, off, M, **kw)   # warm
        sstats = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g = cm.clustermerge_run(res, off, M, **kw)
            sstats.append(g["stats"])
        torch.cuda.synchronize()
        ss_step = (time.perf_counter() - t0) / args.steps
        ss = sstats[-1]
        scr_out = dict(
            time_s=ss_step, speedup_vs_plain=step_s / ss_step, tau=tau, stages="representative and exchange",
            min_product=args.screen_min_product, screen_s=ss["t_screen_s"], screened_pairs=ss["screened_pairs"],
            n_similar_pairs=ss["n_similar_pairs"], screened_out=ss["screened_out"],
            aligned_cells=ss["aligned_cells"], aligned_pairs=ss["aligned_pairs"],
            similar_pairs_vs_plain=ss["n_similar_pairs"] / max(s["n_similar_pairs"], 1),
            calibration=calib, tau_holdout=info["tau"],
            training=dict(workload=f"screen-train: separate 20,000-protein family set (seed 404), "
                                   f"{args.screen_pairs} pairs (half within-family), labels from the GPU "
                                   f"Smith-Waterman (score >= 120), {args.screen_epochs} epochs, batch 4096, "
                                   f"Adam lr 1e-3", gen_s=gen_s, **info))
        if large and not args.no_recall:
            rs = sampled_recall(cm, res, off, M, g["clusters"], ds.n, args.recall_sample)
            scr_out["recall_sample"] = rs
            scr_out["recall"] = rs["recall"]
            scr_out["recall_vs_plain"] = rs["recall"] / max(out["clustermerge"]["recall"], 1e-12)
        elif "truth_pairs" in out["clustermerge"]:
            truth = out["clustermerge"]["truth_pairs"]
            scr_out["recall"] = ss["n_similar_pairs"] / max(truth, 1)
            scr_out["recall_vs_plain"] = scr_out["recall"] / out["clustermerge"]["recall"]
        out["screened"] = scr_out
        log(f"screened: {ss_step:.2f} s/step ({step_s / ss_step:.2f}x), similar pairs "
            f"{ss['n_similar_pairs']} vs {s['n_similar_pairs']}")
        scr.close()

    if not args.no_throughput:
        out["sw_throughput"] = throughput_leg(cm, ctx, args, out, log)

    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
