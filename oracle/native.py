"""ctypes front end of the C oracle (``tc_oracle.c``) -- test infrastructure.

O1 (definition) and O2 (the paper's Procedure 2 + Algorithm 2) run in C
over host threads; the point queries compute single supports and single
vertex triangle counts from their definitions on graphs too large for a
full run in a test.
"""
import ctypes
import os

import numpy as np

from .result import OracleResult

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


class OracleError(RuntimeError):
    pass


def host_threads(cap=16):
    """Threads for a full oracle run: the CPUs this process may use, at most
    ``cap`` (a GPU machine grants one GPU's process 16 host threads)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    return max(1, min(cap, avail))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        common = [_i32p, _i32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int]
        outs = [ctypes.POINTER(ctypes.c_int64), _i32p, _i32p, _u64p, _u64p,
                ctypes.POINTER(ctypes.c_uint64), _u64p, _f64p]
        L.oracle_o1.argtypes = common + outs
        L.oracle_o1.restype = ctypes.c_int
        L.oracle_o2.argtypes = common + [ctypes.c_int32] + outs + [ctypes.c_void_p]
        L.oracle_o2.restype = ctypes.c_int
        L.oracle_query_open.argtypes = [_i32p, _i32p, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_int64)]
        L.oracle_query_open.restype = ctypes.c_int
        L.oracle_query_close.argtypes = [ctypes.c_void_p]
        L.oracle_query_close.restype = None
        L.oracle_query_edges.argtypes = [ctypes.c_void_p, _i32p, _i32p]
        L.oracle_query_degree.argtypes = [ctypes.c_void_p, _i64p]
        L.oracle_query_support.argtypes = [ctypes.c_void_p, _i64p, ctypes.c_int64, _u64p]
        L.oracle_query_tri.argtypes = [ctypes.c_void_p, _i32p, ctypes.c_int64, _u64p]
        for f in (L.oracle_query_edges, L.oracle_query_degree, L.oracle_query_support,
                  L.oracle_query_tri):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _prep(src, dst):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape or src.ndim != 1:
        raise OracleError("src and dst must be 1-D arrays of equal length")
    return src, dst


def _run(which, src, dst, n, nthreads, row_stride=1, phases=None):
    src, dst = _prep(src, dst)
    P = src.shape[0]
    cap = max(P, 1)
    m = ctypes.c_int64(0)
    eu = np.zeros(cap, np.int32)
    ev = np.zeros(cap, np.int32)
    sup = np.zeros(cap, np.uint64)
    tri = np.zeros(max(n, 1), np.uint64)
    triG = ctypes.c_uint64(0)
    num = np.zeros(max(n, 1), np.uint64)
    tc = np.zeros(max(n, 1), np.float64)
    L = lib()
    if which == 1:
        st = L.oracle_o1(src, dst, P, n, nthreads, ctypes.byref(m), eu, ev, sup, tri,
                         ctypes.byref(triG), num, tc)
    else:
        ph = (ctypes.c_double * 4)()
        st = L.oracle_o2(src, dst, P, n, nthreads, row_stride, ctypes.byref(m), eu, ev, sup,
                         tri, ctypes.byref(triG), num, tc, ctypes.cast(ph, ctypes.c_void_p))
        if phases is not None:
            phases.extend(list(ph))
    if st < 0:
        raise OracleError(f"oracle O{which} failed with status {st}")
    mm = m.value
    return OracleResult(n=n, eu=eu[:mm].copy(), ev=ev[:mm].copy(), sup=sup[:mm].copy(),
                        tri=tri[:n].copy(), triG=int(triG.value), num=num[:n].copy(),
                        tc=tc[:n].copy(), status=int(st))


def o1_definition(src, dst, n, nthreads=None):
    """O1: per-edge common neighbours, then Definition 1 (integer form)."""
    return _run(1, src, dst, int(n), nthreads or host_threads())


def o2_paper(src, dst, n, nthreads=None, row_stride=1, phases=None):
    """O2: Procedure 2 with counts + Algorithm 2.

    ``row_stride > 1`` processes only rows v with v % row_stride == 0 in the
    counting loop (a bounded timing sample; its outputs are then partial).
    ``phases`` (a list) receives the seconds spent in normalisation,
    ordering, counting and aggregation.
    """
    return _run(2, src, dst, int(n), nthreads or host_threads(), row_stride, phases)


class PointQuery:
    """Definition-level queries on one normalised graph (no full run)."""

    def __init__(self, src, dst, n):
        src, dst = _prep(src, dst)
        self._h = ctypes.c_void_p()
        m = ctypes.c_int64(0)
        st = lib().oracle_query_open(src, dst, src.shape[0], int(n), ctypes.byref(self._h),
                                     ctypes.byref(m))
        if st < 0:
            raise OracleError(f"oracle_query_open failed with status {st}")
        self.n = int(n)
        self.m = int(m.value)

    def close(self):
        if self._h:
            lib().oracle_query_close(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def edges(self):
        eu = np.zeros(max(self.m, 1), np.int32)
        ev = np.zeros(max(self.m, 1), np.int32)
        lib().oracle_query_edges(self._h, eu, ev)
        return eu[:self.m], ev[:self.m]

    def degree(self):
        d = np.zeros(max(self.n, 1), np.int64)
        lib().oracle_query_degree(self._h, d)
        return d[:self.n]

    def support(self, edge_ids):
        e = np.ascontiguousarray(edge_ids, dtype=np.int64)
        out = np.zeros(max(e.shape[0], 1), np.uint64)
        st = lib().oracle_query_support(self._h, e, e.shape[0], out)
        if st < 0:
            raise OracleError(f"oracle_query_support failed with status {st}")
        return out[:e.shape[0]]

    def tri(self, verts):
        v = np.ascontiguousarray(verts, dtype=np.int32)
        out = np.zeros(max(v.shape[0], 1), np.uint64)
        st = lib().oracle_query_tri(self._h, v, v.shape[0], out)
        if st < 0:
            raise OracleError(f"oracle_query_tri failed with status {st}")
        return out[:v.shape[0]]
