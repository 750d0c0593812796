"""MI355X ClusterMerge hot path: Python binding of libcm.so.

Argument marshalling only: every step of the path runs in the HIP kernels of
``libcm.so`` (see ``include/cm.h`` for the C ABI).  PyTorch supplies device
memory and streams.  There is no CPU fallback: if the library is not built,
importing this package raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1908_10574_amd.build` "
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
_lib.cm_sw_score_batch.restype = _i32
_lib.cm_sw_score_batch.argtypes = [_P, _P, _P, _i32, _P, _i64, _P, _i32, _i32, _P, _P, _P, _P]
_lib.cm_sw_span_batch.restype = _i32
_lib.cm_sw_span_batch.argtypes = [_P, _P, _P, _i32, _P, _i64, _P, _i32, _i32, _P, _P, _P, _i32, _P, _P, _P]

CM_OK, CM_EINVAL, CM_ERANGE, CM_ENOMEM, CM_EDEVICE, CM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
CM_MAX_LEN = 16384


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


def sync(ctx: Context | None = None):
    (ctx or context()).sync()
