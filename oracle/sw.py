"""ctypes loader for the scalar C oracle (``sw_oracle.c``). Test infrastructure only."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib_path() -> str:
    return os.path.join(_HERE, "liboracle_sw.so")


def _lib():
    global _LIB
    if _LIB is None:
        path = lib_path()
        if not os.path.exists(path):
            from .build_oracle import build
            build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.oracle_sw.restype = i32
        L.oracle_sw.argtypes = [P, i32, P, i32, P, i32, i32, P, P]
        L.oracle_sw_span.restype = i32
        L.oracle_sw_span.argtypes = [P, i32, P, i32, P, i32, i32, P]
        L.oracle_sw_batch.restype = None
        L.oracle_sw_batch.argtypes = [P, P, P, i64, P, i32, i32, P, P, P]
        L.oracle_span_batch.restype = i64
        L.oracle_span_batch.argtypes = [P, P, P, i64, P, i32, i32, P]
        L.oracle_traceback_batch.restype = i64
        L.oracle_traceback_batch.argtypes = [P, P, P, i64, P, i32, i32, P, P, P, P]
        _LIB = L
    return _LIB


def _u8(x):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.uint8))
    return x, x.ctypes.data if len(x) else None


def _mat(M):
    M = np.ascontiguousarray(np.asarray(M, dtype=np.int32).reshape(20, 20))
    return M


def sw(a, b, M, go=-11, ge=-1):
    """(score, end_i, end_j) of one pair; a gives rows, b columns."""
    a, pa = _u8(a)
    b, pb = _u8(b)
    M = _mat(M)
    ei, ej = ctypes.c_int32(), ctypes.c_int32()
    s = _lib().oracle_sw(pa, len(a), pb, len(b), M.ctypes.data, go, ge,
                         ctypes.byref(ei), ctypes.byref(ej))
    return int(s), ei.value, ej.value


def sw_span(a, b, M, go=-11, ge=-1):
    """(score, end_i, end_j, start_i, start_j) of one pair."""
    a, pa = _u8(a)
    b, pb = _u8(b)
    M = _mat(M)
    out = np.zeros(5, np.int32)
    rc = _lib().oracle_sw_span(pa, len(a), pb, len(b), M.ctypes.data, go, ge, out.ctypes.data)
    if rc != 0:
        raise AssertionError("oracle reverse pass did not reproduce the score")
    return tuple(int(v) for v in out)


def sw_batch(residues, offsets, pairs, M, go=-11, ge=-1, with_end=True):
    """Scores (and end cells) of every pair row (a, b); single-threaded."""
    res = np.ascontiguousarray(residues, dtype=np.uint8)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    M = _mat(M)
    n = len(pr)
    sc = np.zeros(n, np.int32)
    ea = np.zeros(n, np.int32) if with_end else None
    eb = np.zeros(n, np.int32) if with_end else None
    if n:
        _lib().oracle_sw_batch(res.ctypes.data if len(res) else None, off.ctypes.data,
                               pr.ctypes.data, n, M.ctypes.data, go, ge, sc.ctypes.data,
                               ea.ctypes.data if with_end else None,
                               eb.ctypes.data if with_end else None)
    return (sc, ea, eb) if with_end else sc


def span_batch(residues, offsets, pairs, M, go=-11, ge=-1):
    """[n][5] = score, end_a, end_b, start_a, start_b for every pair row."""
    res = np.ascontiguousarray(residues, dtype=np.uint8)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    M = _mat(M)
    out = np.zeros((len(pr), 5), np.int32)
    if len(pr):
        bad = _lib().oracle_span_batch(res.ctypes.data if len(res) else None, off.ctypes.data,
                                       pr.ctypes.data, len(pr), M.ctypes.data, go, ge,
                                       out.ctypes.data)
        if bad:
            raise AssertionError(f"oracle reverse pass failed on {bad} pairs")
    return out


def traceback_batch(residues, offsets, pairs, M, go=-11, ge=-1, span=None):
    """Alignment columns ('M', 'I', 'D', start to end) of each pair's optimal
    local alignment between its start and end cells (``sw_oracle.c``,
    oracle_sw_traceback).  span: the [n][5] rows of span_batch (computed when
    None).  Returns (list of str, span rows)."""
    res = np.ascontiguousarray(residues, dtype=np.uint8)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    if span is None:
        span = span_batch(res, off, pr, M, go, ge)
    span = np.ascontiguousarray(span, dtype=np.int32)
    cap = np.where(span[:, 0] > 0, (span[:, 1] - span[:, 3] + 1) + (span[:, 2] - span[:, 4] + 1), 0)
    op_off = np.zeros(len(pr) + 1, np.int64)
    np.cumsum(cap, out=op_off[1:])
    ops = np.zeros(max(int(op_off[-1]), 1), np.uint8)
    n_ops = np.zeros(len(pr), np.int32)
    if len(pr):
        bad = _lib().oracle_traceback_batch(res.ctypes.data if len(res) else None, off.ctypes.data,
                                            pr.ctypes.data, len(pr), _mat(M).ctypes.data, go, ge,
                                            span.ctypes.data, op_off.ctypes.data, ops.ctypes.data,
                                            n_ops.ctypes.data)
        if bad:
            raise AssertionError(f"oracle traceback failed on {bad} pairs")
    out = [bytes(ops[op_off[p]:op_off[p] + n_ops[p]]).decode() for p in range(len(pr))]
    return out, span
