"""MI355X ClusterMerge hot path: Python binding of libcm.so.

Argument marshalling only: every step of the path runs in the HIP kernels of
``libcm.so`` (see ``include/cm.h`` for the C ABI).  PyTorch supplies device
memory and streams.  There is no CPU fallback: if the library is not built,
importing this package raises.

Entry points: ``sw_score_batch`` (score, end cell), ``sw_span_batch`` (start
cell), ``sw_traceback_batch`` (alignment columns), ``clustermerge_run``,
``clustermerge_extend`` (new proteins against a previous clustering),
``allvsall_count``, ``kmer_features`` and the ``Screen`` (learned pair screen:
inference and training), ``Context`` (plans, autotuning, graphs, timing).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python {os.path.join(_HERE, 'build.py')}` "
                      "(hipcc, gfx950); there is no fallback path")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_i32, _i64, _u64, _f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float

_lib.cm_status_str.restype = ctypes.c_char_p
_lib.cm_status_str.argtypes = [_i32]
_lib.cm_last_error.restype = ctypes.c_char_p
_lib.cm_last_error.argtypes = []
_lib.cm_context_create.restype = _i32
_lib.cm_context_create.argtypes = [ctypes.c_int, ctypes.POINTER(_P)]
_lib.cm_context_destroy.restype = None
_lib.cm_context_destroy.argtypes = [_P]
_lib.cm_context_sync.restype = _i32
_lib.cm_context_sync.argtypes = [_P]
_lib.cm_context_set_timing.restype = _i32
_lib.cm_context_set_timing.argtypes = [_P, ctypes.c_int]
_lib.cm_context_set_graphs.restype = _i32
_lib.cm_context_set_graphs.argtypes = [_P, ctypes.c_int]
_lib.cm_context_kernel_time.restype = _i32
_lib.cm_context_kernel_time.argtypes = [_P, ctypes.c_int, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double)]
_lib.cm_context_cells_computed.restype = _i32
_lib.cm_context_cells_computed.argtypes = [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
_lib.cm_plan_get.restype = _i32
_lib.cm_plan_get.argtypes = [_P, ctypes.c_int, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                             ctypes.POINTER(_i32)]
_lib.cm_plan_set.restype = _i32
_lib.cm_plan_set.argtypes = [_P, ctypes.c_int, _i32, _i32, _i32]
_lib.cm_plan_save.restype = _i32
_lib.cm_plan_save.argtypes = [_P, ctypes.c_char_p]
_lib.cm_plan_load.restype = _i32
_lib.cm_plan_load.argtypes = [_P, ctypes.c_char_p]
_lib.cm_autotune.restype = _i32
_lib.cm_autotune.argtypes = [_P, _P, _P, _i32, _P, _i64, _P, _i32, _i32, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32)]
_lib.cm_sw_score_batch.restype = _i32
_lib.cm_sw_score_batch.argtypes = [_P, _P, _P, _i32, _P, _i64, _P, _i32, _i32, _P, _P, _P, _P]
_lib.cm_sw_span_batch.restype = _i32
_lib.cm_sw_span_batch.argtypes = [_P, _P, _P, _i32, _P, _i64, _P, _i32, _i32, _P, _P, _P, _i32, _P, _P, _P]


class CMParams(ctypes.Structure):
    _fields_ = [("matrix", _i32 * 400), ("gap_open", _i32), ("gap_extend", _i32), ("T", _i32),
                ("mT", _i32), ("mU", _i32), ("screen_stages", ctypes.c_uint32), ("screen_tau", _f32),
                ("max_result_pairs", _i64), ("screen_min_product", _i64), ("rep_chunk_pairs", _i64),
                ("record_candidates", _i64)]


class CMStats(ctypes.Structure):
    _fields_ = [("rep_comparisons", _i64), ("exchange_alignments", _i64), ("full_merges", _i64),
                ("exchanges", _i64), ("rounds", _i64), ("waves", _i64), ("aligned_pairs", _i64),
                ("aligned_cells", ctypes.c_double), ("speculative_pairs", _i64), ("cache_hits", _i64),
                ("screened_out", _i64), ("n_clusters", _i64), ("final_candidates", _i64),
                ("n_similar_pairs", _i64), ("pair_set_hash", _u64), ("t_total_s", ctypes.c_double),
                ("t_merge_s", ctypes.c_double), ("t_final_s", ctypes.c_double), ("t_gpu_s", ctypes.c_double),
                ("t_host_s", ctypes.c_double), ("sw_launches", _i64), ("sw_kernel_s", ctypes.c_double),
                ("end_kernel_s", ctypes.c_double), ("end_pairs", _i64),
                ("t_screen_s", ctypes.c_double), ("screened_pairs", _i64), ("required_cells", ctypes.c_double)]


_lib.cm_clustermerge_run.restype = _i32
_lib.cm_clustermerge_run.argtypes = [_P, _P, _P, _i32, ctypes.POINTER(CMParams), _P, ctypes.POINTER(_P)]
_lib.cm_sw_traceback_batch.restype = _i32
_lib.cm_sw_traceback_batch.argtypes = [_P, _P, _P, _i32, _P, _i64, _P, _i32, _i32, _P, _P, _P, _P, _P, _P, _P, _P,
                                       _P]
_lib.cm_clustermerge_extend.restype = _i32
_lib.cm_clustermerge_extend.argtypes = [_P, _P, _P, _i32, ctypes.POINTER(CMParams), _P, _i32, _i32, _P, _P, _P,
                                        _i64, _P, _P, ctypes.POINTER(_P)]
_lib.cm_result_clusters.restype = _i32
_lib.cm_result_clusters.argtypes = [_P, ctypes.POINTER(_i32), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                    ctypes.POINTER(_P)]
_lib.cm_result_pairs.restype = _i32
_lib.cm_result_pairs.argtypes = [_P, ctypes.POINTER(_i64), ctypes.POINTER(_P), ctypes.POINTER(_P)]
_lib.cm_result_candidates.restype = _i32
_lib.cm_result_candidates.argtypes = [_P, ctypes.POINTER(_i64), ctypes.POINTER(_P), ctypes.POINTER(_P)]
_lib.cm_result_stats.restype = _i32
_lib.cm_result_stats.argtypes = [_P, ctypes.POINTER(CMStats)]
_lib.cm_result_free.restype = None
_lib.cm_result_free.argtypes = [_P]
_lib.cm_allvsall_count.restype = _i32
_lib.cm_allvsall_count.argtypes = [_P, _P, _P, _i32, _P, _i32, _i32, _i32, ctypes.POINTER(_i64),
                                   ctypes.POINTER(ctypes.c_double)]

_lib.cm_probe_valu.restype = _i32
_lib.cm_probe_valu.argtypes = [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]

CM_STAGE_REP, CM_STAGE_EXCHANGE, CM_STAGE_FINAL = 1, 2, 4
CM_PROBE_I32_ADD, CM_PROBE_I32_MAX3, CM_PROBE_PK16_ADD, CM_PROBE_PK16_MAX3 = 0, 1, 2, 3


def probe_valu(kind: int, ctx: "Context | None" = None):
    """(operations per second, shader clock in Hz) of one VALU instruction at
    full occupancy (cm_probe_valu); packed 16-bit halves count as two."""
    ctx = ctx or context()
    ops, clk = ctypes.c_double(), ctypes.c_double()
    _check(_lib.cm_probe_valu(ctx.handle, int(kind), ctypes.byref(ops), ctypes.byref(clk)))
    return ops.value, clk.value

CM_OK, CM_EINVAL, CM_ERANGE, CM_ENOMEM, CM_EDEVICE, CM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
CM_MAX_LEN = 65535


class CMError(RuntimeError):
    def __init__(self, status: int):
        self.status = status
        msg = _lib.cm_last_error().decode(errors="replace")
        super().__init__(f"{_lib.cm_status_str(status).decode()} ({status}): {msg}")


def _check(status: int):
    if status != CM_OK:
        raise CMError(status)


def lib():
    """The loaded ctypes library (for tests of the raw ABI)."""
    return _lib


class Context:
    """Owns a cm_context (device scratch, persistent-grid sizes, error flag)."""

    def __init__(self, device: int = 0):
        h = _P()
        _check(_lib.cm_context_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            _lib.cm_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(_lib.cm_context_sync(self.handle))

    def set_graphs(self, on: bool):
        """Replay ClusterMerge waves as captured hipGraphs."""
        _check(_lib.cm_context_set_graphs(self.handle, int(bool(on))))

    def set_timing(self, on: bool):
        _check(_lib.cm_context_set_timing(self.handle, int(bool(on))))

    def get_plan(self, pass_: int):
        """(packed, rmax, blocks_per_cu, max_blocks_per_cu) of a pass (0 score, 1 score+end, 2 span)."""
        k, r, b, m = _i32(), _i32(), _i32(), _i32()
        _check(_lib.cm_plan_get(self.handle, int(pass_), ctypes.byref(k), ctypes.byref(r), ctypes.byref(b),
                                ctypes.byref(m)))
        return k.value, r.value, b.value, m.value

    def set_plan(self, pass_: int, packed: int, rmax: int, blocks_per_cu: int):
        _check(_lib.cm_plan_set(self.handle, int(pass_), int(packed), int(rmax), int(blocks_per_cu)))

    def save_plans(self, path: str):
        _check(_lib.cm_plan_save(self.handle, str(path).encode()))

    def load_plans(self, path: str):
        _check(_lib.cm_plan_load(self.handle, str(path).encode()))

    def autotune(self, residues, offsets, pairs, matrix, pass_: int = 0, gap_open: int = -11,
                 gap_extend: int = -1):
        """Time every candidate plan on a pair sample; keeps the fastest.  Returns rows
        (packed, rmax, blocks_per_cu, ms)."""
        import torch
        residues = _dev(residues, torch.uint8, "residues")
        offsets = _dev(offsets, torch.int64, "offsets")
        pairs = _dev(pairs, torch.int32, "pairs")
        torch.cuda.current_stream().synchronize()
        tab = (ctypes.c_double * 128)()
        n = _i32()
        m = _matrix_host(matrix)
        _check(_lib.cm_autotune(self.handle, residues.data_ptr() if residues.numel() else None,
                                offsets.data_ptr(), offsets.numel() - 1, pairs.data_ptr(), pairs.numel() // 2,
                                m.ctypes.data, int(gap_open), int(gap_extend), int(pass_), tab, ctypes.byref(n)))
        return [(int(tab[4 * k]), int(tab[4 * k + 1]), int(tab[4 * k + 2]), float(tab[4 * k + 3]))
                for k in range(n.value)]

    def kernel_time(self, pass_: int):
        """(launches, seconds) of alignment-kernel launches timed so far for a pass
        (0 score, 1 score+end, 2 span)."""
        n, sec = _i64(), ctypes.c_double()
        _check(_lib.cm_context_kernel_time(self.handle, int(pass_), ctypes.byref(n), ctypes.byref(sec)))
        return n.value, sec.value

    def cells_computed(self, pass_: int) -> float:
        """DP cells the alignment kernels of a pass computed in timed launches so far
        (ramps and padding included)."""
        c = ctypes.c_double()
        _check(_lib.cm_context_cells_computed(self.handle, int(pass_), ctypes.byref(c)))
        return c.value


_default_ctx: Context | None = None


def context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        import torch
        _default_ctx = Context(torch.cuda.current_device())
    return _default_ctx


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _matrix_host(matrix):
    m = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32).reshape(400))
    return m


def sw_score_batch(residues, offsets, pairs, matrix, gap_open: int = -11, gap_extend: int = -1,
                   return_end: bool = False, ctx: Context | None = None, stream=None, out=None):
    """Smith-Waterman scores (and end cells) of every pair row (a, b).

    residues u8, offsets i64 [n+1], pairs i32 [P, 2]: CUDA tensors.  matrix: 20x20
    host ints.  Returns int32 CUDA tensors: scores, or (scores, end_a, end_b).
    Work is enqueued on the current (or given) stream; nothing is synchronized.
    """
    import torch
    ctx = ctx or context()
    residues = _dev(residues, torch.uint8, "residues")
    offsets = _dev(offsets, torch.int64, "offsets")
    pairs = _dev(pairs, torch.int32, "pairs")
    n_pairs = pairs.numel() // 2
    dev = pairs.device
    if out is None:
        scores = torch.empty(n_pairs, dtype=torch.int32, device=dev)
        ea = torch.empty(n_pairs, dtype=torch.int32, device=dev) if return_end else None
        eb = torch.empty(n_pairs, dtype=torch.int32, device=dev) if return_end else None
    else:
        scores, ea, eb = out
    m = _matrix_host(matrix)
    _check(_lib.cm_sw_score_batch(ctx.handle, residues.data_ptr() if residues.numel() else None,
                                  offsets.data_ptr(), offsets.numel() - 1, pairs.data_ptr(), n_pairs,
                                  m.ctypes.data, int(gap_open), int(gap_extend), scores.data_ptr(),
                                  ea.data_ptr() if ea is not None else None,
                                  eb.data_ptr() if eb is not None else None, _stream_ptr(stream)))
    return (scores, ea, eb) if return_end else scores


def sw_span_batch(residues, offsets, pairs, matrix, scores, end_a, end_b, min_score: int = 0,
                  gap_open: int = -11, gap_extend: int = -1, ctx: Context | None = None, stream=None):
    """Start cells of the optimal alignments of pairs whose score exceeds min_score."""
    import torch
    ctx = ctx or context()
    residues = _dev(residues, torch.uint8, "residues")
    offsets = _dev(offsets, torch.int64, "offsets")
    pairs = _dev(pairs, torch.int32, "pairs")
    n_pairs = pairs.numel() // 2
    sa = torch.empty(n_pairs, dtype=torch.int32, device=pairs.device)
    sb = torch.empty(n_pairs, dtype=torch.int32, device=pairs.device)
    m = _matrix_host(matrix)
    _check(_lib.cm_sw_span_batch(ctx.handle, residues.data_ptr() if residues.numel() else None,
                                 offsets.data_ptr(), offsets.numel() - 1, pairs.data_ptr(), n_pairs,
                                 m.ctypes.data, int(gap_open), int(gap_extend), scores.data_ptr(),
                                 end_a.data_ptr(), end_b.data_ptr(), int(min_score), sa.data_ptr(),
                                 sb.data_ptr(), _stream_ptr(stream)))
    return sa, sb


def sw_traceback_batch(residues, offsets, pairs, matrix, scores, end_a, end_b, start_a, start_b,
                       gap_open: int = -11, gap_extend: int = -1, ctx: Context | None = None, stream=None):
    """Alignment columns ('M', 'I', 'D', start to end) of the pairs' optimal
    local alignments between their start and end cells.  Returns (ops u8,
    op_offsets i64 [n+1], n_ops i32) as tensors on the pairs' device; pair p's
    columns are ops[op_offsets[p] : op_offsets[p] + n_ops[p]]."""
    import torch
    ctx = ctx or context()
    residues = _dev(residues, torch.uint8, "residues")
    offsets = _dev(offsets, torch.int64, "offsets")
    pairs = _dev(pairs, torch.int32, "pairs")
    n_pairs = pairs.numel() // 2
    cap = torch.where(scores > 0, (end_a - start_a + 1) + (end_b - start_b + 1), torch.zeros_like(scores))
    op_off = torch.zeros(n_pairs + 1, dtype=torch.int64, device=pairs.device)
    if n_pairs:
        op_off[1:] = torch.cumsum(cap.clamp(min=0).to(torch.int64), 0)
    ops = torch.zeros(max(int(op_off[-1].item()), 1), dtype=torch.uint8, device=pairs.device)
    n_ops = torch.zeros(n_pairs, dtype=torch.int32, device=pairs.device)
    m = _matrix_host(matrix)
    _check(_lib.cm_sw_traceback_batch(ctx.handle, residues.data_ptr() if residues.numel() else None,
                                      offsets.data_ptr(), offsets.numel() - 1, pairs.data_ptr(), n_pairs,
                                      m.ctypes.data, int(gap_open), int(gap_extend), scores.data_ptr(),
                                      end_a.data_ptr(), end_b.data_ptr(), start_a.data_ptr(), start_b.data_ptr(),
                                      op_off.data_ptr(), ops.data_ptr(), n_ops.data_ptr(), _stream_ptr(stream)))
    return ops, op_off, n_ops


def columns_as_strings(ops, op_off, n_ops):
    """Host strings of sw_traceback_batch's output."""
    o = ops.cpu().numpy()
    off = op_off.cpu().numpy()
    n = n_ops.cpu().numpy()
    return [bytes(o[off[p]:off[p] + max(n[p], 0)]).decode() for p in range(len(n))]


def sync(ctx: Context | None = None):
    (ctx or context()).sync()


def _np_from(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype=dtype)
    ct = {np.int32: _i32, np.int64: _i64}[dtype]
    return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ct)), shape=(n,)).copy()


def make_params(matrix, T=120, mT=166, mU=15, gap_open=-11, gap_extend=-1, screen_stages=0,
                screen_tau=0.0, max_result_pairs=1 << 62, screen_min_product=0, rep_chunk_pairs=0,
                record_candidates=False) -> CMParams:
    p = CMParams()
    m = _matrix_host(matrix)
    for k in range(400):
        p.matrix[k] = int(m[k])
    p.gap_open, p.gap_extend, p.T, p.mT, p.mU = int(gap_open), int(gap_extend), int(T), int(mT), int(mU)
    p.screen_stages, p.screen_tau, p.max_result_pairs = int(screen_stages), float(screen_tau), int(max_result_pairs)
    p.screen_min_product = int(screen_min_product)
    p.rep_chunk_pairs = int(rep_chunk_pairs)
    p.record_candidates = 1 if record_candidates else 0
    return p


def clustermerge_run(residues, offsets, matrix, T=120, mT=166, mU=15, gap_open=-11, gap_extend=-1,
                     screen=None, screen_stages=CM_STAGE_REP | CM_STAGE_EXCHANGE, screen_tau=0.0,
                     max_result_pairs=1 << 62, screen_min_product=0, rep_chunk_pairs=0,
                     record_candidates=False, ctx: Context | None = None):
    """ClusterMerge on a device-resident store (residues u8, offsets i64: CUDA tensors).

    Returns dict(clusters=[(rep, members ndarray)], pairs=ndarray [k,2], scores=ndarray [k],
    stats=dict), and with record_candidates also candidates=ndarray [c,2] and
    candidate_scores=ndarray [c] (the pairs scored during the merge stage).  Synchronous.
    """
    import torch
    ctx = ctx or context()
    residues = _dev(residues, torch.uint8, "residues")
    offsets = _dev(offsets, torch.int64, "offsets")
    torch.cuda.current_stream().synchronize()
    p = make_params(matrix, T, mT, mU, gap_open, gap_extend, screen_stages if screen else 0, screen_tau,
                    max_result_pairs, screen_min_product, rep_chunk_pairs, record_candidates)
    res = _P()
    _check(_lib.cm_clustermerge_run(ctx.handle, residues.data_ptr() if residues.numel() else None,
                                    offsets.data_ptr(), offsets.numel() - 1, ctypes.byref(p),
                                    screen.handle if screen is not None else None, ctypes.byref(res)))
    return _take_result(res)


def _take_result(res):
    """Copy a library-owned cm_result into Python objects and free it."""
    try:
        nc = _i32()
        reps, moff, mem = _P(), _P(), _P()
        _check(_lib.cm_result_clusters(res, ctypes.byref(nc), ctypes.byref(reps), ctypes.byref(moff),
                                       ctypes.byref(mem)))
        reps_a = _np_from(reps.value, nc.value, np.int32)
        moff_a = _np_from(moff.value, nc.value + 1, np.int64)
        mem_a = _np_from(mem.value, int(moff_a[-1]) if len(moff_a) else 0, np.int32)
        clusters = [(int(reps_a[k]), mem_a[moff_a[k]:moff_a[k + 1]]) for k in range(nc.value)]
        npr = _i64()
        pp, ps = _P(), _P()
        _check(_lib.cm_result_pairs(res, ctypes.byref(npr), ctypes.byref(pp), ctypes.byref(ps)))
        pairs = _np_from(pp.value, 2 * npr.value, np.int32).reshape(-1, 2)
        scores = _np_from(ps.value, npr.value, np.int32)
        st = CMStats()
        _check(_lib.cm_result_stats(res, ctypes.byref(st)))
        stats = {k: getattr(st, k) for k, _ in CMStats._fields_}
        nc2 = _i64()
        cp, cs = _P(), _P()
        _check(_lib.cm_result_candidates(res, ctypes.byref(nc2), ctypes.byref(cp), ctypes.byref(cs)))
        extra = {}
        if nc2.value:
            extra = dict(candidates=_np_from(cp.value, 2 * nc2.value, np.int32).reshape(-1, 2),
                         candidate_scores=_np_from(cs.value, nc2.value, np.int32))
    finally:
        _lib.cm_result_free(res)
    return dict(clusters=clusters, pairs=pairs, scores=scores, stats=stats, **extra)


def clustermerge_extend(residues, offsets, matrix, prev_clusters, n_prev, known_pairs=None, known_scores=None,
                        T=120, mT=166, mU=15, gap_open=-11, gap_extend=-1, screen=None,
                        screen_stages=CM_STAGE_REP | CM_STAGE_EXCHANGE, screen_tau=0.0, max_result_pairs=1 << 62,
                        screen_min_product=0, rep_chunk_pairs=0, ctx: Context | None = None):
    """Classify proteins n_prev.. of the store against a previous clustering of
    proteins 0..n_prev-1 (prev_clusters: [(rep, members)], e.g. the "clusters"
    of a clustermerge_run result); known_pairs [k,2] / known_scores [k] (e.g.
    its "pairs" / "scores") are reused.  Returns the same dict as
    clustermerge_run.  Synchronous."""
    import torch
    ctx = ctx or context()
    residues = _dev(residues, torch.uint8, "residues")
    offsets = _dev(offsets, torch.int64, "offsets")
    torch.cuda.current_stream().synchronize()
    p = make_params(matrix, T, mT, mU, gap_open, gap_extend, screen_stages if screen else 0, screen_tau,
                    max_result_pairs, screen_min_product, rep_chunk_pairs)
    reps = np.ascontiguousarray([int(r) for r, _ in prev_clusters], dtype=np.int32)
    sizes = np.array([len(m) for _, m in prev_clusters], dtype=np.int64)
    moff = np.zeros(len(prev_clusters) + 1, dtype=np.int64)
    np.cumsum(sizes, out=moff[1:])
    mem = (np.ascontiguousarray(np.concatenate([np.asarray(m, np.int32) for _, m in prev_clusters]))
           if len(prev_clusters) else np.zeros(1, np.int32))
    kp = np.ascontiguousarray(known_pairs if known_pairs is not None else np.zeros((0, 2)), dtype=np.int32)
    ks = np.ascontiguousarray(known_scores if known_scores is not None else np.zeros(0), dtype=np.int32)
    if len(kp) != len(ks):
        raise ValueError("known_pairs and known_scores differ in length")
    res = _P()
    _check(_lib.cm_clustermerge_extend(ctx.handle, residues.data_ptr() if residues.numel() else None,
                                       offsets.data_ptr(), offsets.numel() - 1, ctypes.byref(p),
                                       screen.handle if screen is not None else None, int(n_prev),
                                       len(prev_clusters), reps.ctypes.data, moff.ctypes.data, mem.ctypes.data,
                                       len(ks), kp.ctypes.data if len(kp) else None,
                                       ks.ctypes.data if len(ks) else None, ctypes.byref(res)))
    return _take_result(res)


def allvsall_count(residues, offsets, matrix, T=120, gap_open=-11, gap_extend=-1, ctx: Context | None = None):
    """(count of pairs x < y with score >= T over the whole store, cells aligned)."""
    import torch
    ctx = ctx or context()
    residues = _dev(residues, torch.uint8, "residues")
    offsets = _dev(offsets, torch.int64, "offsets")
    torch.cuda.current_stream().synchronize()
    m = _matrix_host(matrix)
    cnt, cells = _i64(), ctypes.c_double()
    _check(_lib.cm_allvsall_count(ctx.handle, residues.data_ptr() if residues.numel() else None,
                                  offsets.data_ptr(), offsets.numel() - 1, m.ctypes.data, int(gap_open),
                                  int(gap_extend), int(T), ctypes.byref(cnt), ctypes.byref(cells)))
    return cnt.value, cells.value


# ---------------------------------------------------------------------------
# learned pair screen
# ---------------------------------------------------------------------------
_lib.cm_kmer_features.restype = _i32
_lib.cm_kmer_features.argtypes = [_P, _P, _P, _i32, _P, _P]
_lib.cm_screen_num_params.restype = _i64
_lib.cm_screen_num_params.argtypes = []
_lib.cm_screen_create.restype = _i32
_lib.cm_screen_create.argtypes = [_P, _u64, ctypes.POINTER(_P)]
_lib.cm_screen_destroy.restype = None
_lib.cm_screen_destroy.argtypes = [_P]
_lib.cm_screen_set_weights.restype = _i32
_lib.cm_screen_set_weights.argtypes = [_P, _P]
_lib.cm_screen_get_weights.restype = _i32
_lib.cm_screen_get_weights.argtypes = [_P, _P, _P]
_lib.cm_screen_infer.restype = _i32
_lib.cm_screen_infer.argtypes = [_P, _P, _P, _i64, _P, _P]
_lib.cm_screen_grads.restype = _i32
_lib.cm_screen_grads.argtypes = [_P, _P, _P, _P, _i64, _P, ctypes.POINTER(_f32)]
_lib.cm_screen_train_step.restype = _i32
_lib.cm_screen_train_step.argtypes = [_P, _P, _P, _P, _i64, _f32, ctypes.POINTER(_f32)]


class CMTrainCfg(ctypes.Structure):
    _fields_ = [("epochs", _i32), ("batch", _i32), ("lr", _f32), ("shuffle", _i32), ("seed", _u64),
                ("drop_last", _i32)]


_lib.cm_screen_train_steps.restype = _i64
_lib.cm_screen_train_steps.argtypes = [_i64, ctypes.POINTER(CMTrainCfg)]
_lib.cm_screen_train.restype = _i32
_lib.cm_screen_train.argtypes = [_P, _P, _P, _P, _i64, ctypes.POINTER(CMTrainCfg), _P]
_lib.cm_screen_save.restype = _i32
_lib.cm_screen_save.argtypes = [_P, ctypes.c_char_p]
_lib.cm_screen_load.restype = _i32
_lib.cm_screen_load.argtypes = [_P, ctypes.c_char_p, ctypes.POINTER(_P)]

SCREEN_PARAMS = int(_lib.cm_screen_num_params())


def kmer_features(residues, offsets, ctx: Context | None = None, stream=None):
    """Hashed 3-mer count features, bf16 CUDA tensor [n_seqs][1024]."""
    import torch
    ctx = ctx or context()
    residues = _dev(residues, torch.uint8, "residues")
    offsets = _dev(offsets, torch.int64, "offsets")
    n = offsets.numel() - 1
    feat = torch.empty((max(n, 0), 1024), dtype=torch.bfloat16, device=offsets.device)
    _check(_lib.cm_kmer_features(ctx.handle, residues.data_ptr() if residues.numel() else None,
                                 offsets.data_ptr(), n, feat.data_ptr(), _stream_ptr(stream)))
    return feat


class Screen:
    """The MLP pair screen (weights, Adam state and workspace on the device)."""

    def __init__(self, seed: int = 0, ctx: Context | None = None, _handle=None):
        self.ctx = ctx or context()
        if _handle is None:
            h = _P()
            _check(_lib.cm_screen_create(self.ctx.handle, int(seed), ctypes.byref(h)))
            _handle = h
        self.handle = _handle

    @classmethod
    def load(cls, path: str, ctx: Context | None = None) -> "Screen":
        ctx = ctx or context()
        h = _P()
        _check(_lib.cm_screen_load(ctx.handle, str(path).encode(), ctypes.byref(h)))
        return cls(ctx=ctx, _handle=h)

    def close(self):
        if getattr(self, "handle", None):
            _lib.cm_screen_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def save(self, path: str):
        _check(_lib.cm_screen_save(self.handle, str(path).encode()))

    def set_weights(self, master):
        m = np.ascontiguousarray(np.asarray(master, dtype=np.float32).reshape(-1))
        if m.size != SCREEN_PARAMS:
            raise ValueError(f"expected {SCREEN_PARAMS} parameters, got {m.size}")
        _check(_lib.cm_screen_set_weights(self.handle, m.ctypes.data))

    def get_weights(self):
        """(fp32 master [num_params], bf16 bit patterns of W1|W2|W3 as uint16)."""
        m = np.zeros(SCREEN_PARAMS, np.float32)
        b = np.zeros(512 * 2048 + 512 * 512 + 512, np.uint16)
        _check(_lib.cm_screen_get_weights(self.handle, m.ctypes.data, b.ctypes.data))
        return m, b

    def infer(self, feat, pairs, stream=None):
        import torch
        pairs = _dev(pairs, torch.int32, "pairs")
        n = pairs.numel() // 2
        out = torch.empty(n, dtype=torch.float32, device=pairs.device)
        if n:
            _check(_lib.cm_screen_infer(self.handle, feat.data_ptr(), pairs.data_ptr(), n, out.data_ptr(),
                                        _stream_ptr(stream)))
        return out

    def grads(self, feat, pairs, labels):
        import torch
        torch.cuda.current_stream().synchronize()
        pairs = _dev(pairs, torch.int32, "pairs")
        labels = _dev(labels, torch.uint8, "labels")
        g = np.zeros(SCREEN_PARAMS, np.float32)
        loss = _f32()
        _check(_lib.cm_screen_grads(self.handle, feat.data_ptr(), pairs.data_ptr(), labels.data_ptr(),
                                    pairs.numel() // 2, g.ctypes.data, ctypes.byref(loss)))
        return g, loss.value

    def train(self, feat, pairs, labels, epochs: int = 5, batch: int = 4096, lr: float = 1e-3,
              shuffle: bool = True, seed: int = 0, drop_last: bool = True) -> np.ndarray:
        """A whole training run on the device (cm_screen_train); returns the
        per-step mean loss log (numpy float32, one entry per Adam step)."""
        import torch
        torch.cuda.current_stream().synchronize()
        pairs = _dev(pairs, torch.int32, "pairs")
        labels = _dev(labels, torch.uint8, "labels")
        cfg = CMTrainCfg(int(epochs), int(batch), float(lr), int(bool(shuffle)), int(seed), int(bool(drop_last)))
        n = pairs.numel() // 2
        steps = _lib.cm_screen_train_steps(n, ctypes.byref(cfg))
        if steps < 1:
            raise ValueError(f"training config makes no step ({steps}) for {n} pairs")
        log = np.zeros(steps, np.float32)
        _check(_lib.cm_screen_train(self.handle, feat.data_ptr(), pairs.data_ptr(), labels.data_ptr(), n,
                                    ctypes.byref(cfg), log.ctypes.data))
        return log

    def train_step(self, feat, pairs, labels, lr: float = 1e-3) -> float:
        import torch
        torch.cuda.current_stream().synchronize()
        pairs = _dev(pairs, torch.int32, "pairs")
        labels = _dev(labels, torch.uint8, "labels")
        loss = _f32()
        _check(_lib.cm_screen_train_step(self.handle, feat.data_ptr(), pairs.data_ptr(), labels.data_ptr(),
                                         pairs.numel() // 2, float(lr), ctypes.byref(loss)))
        return loss.value
