"""Thin ctypes binding of libtc (the C ABI in include/tc.h).

The functions named ``tc_*`` here mirror the C entry points one to one and
only marshal arguments: every step of the computation runs in libtc's HIP
kernels.  Buffers are passed as raw pointers: device buffers are torch CUDA
tensors (PyTorch only allocates memory and provides the stream), host
buffers are numpy arrays.  There is no fallback: if libtc.so is missing or
fails to load, every call raises.

``Graph`` wraps a handle for convenience (tests, benchmark, server).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc.so")

TC_OK = 0
TC_TRIANGLE_FREE = 1
TC_ERR_INVALID_ARG = -1
TC_ERR_VERTEX_RANGE = -2
TC_ERR_OOM = -3
TC_ERR_DEVICE = -4
TC_ERR_OVERFLOW = -5
TC_ERR_BUDGET = -6
TC_ERR_NOT_COMPUTED = -7
TC_ERR_UNSUPPORTED = -8
TC_ERR_IO = -9

TC_MEM_HOST = 0
TC_MEM_DEVICE = 1

TC_ALGO_AUTO = 0
TC_ALGO_LOW_PIVOT = 1
TC_ALGO_MID_PIVOT = 2

_lib = None


class TCError(RuntimeError):
    def __init__(self, status, where):
        self.status = int(status)
        msg = _lib.tc_status_string(int(status)).decode() if _lib else str(status)
        super().__init__(f"{where}: {msg} (status {status})")


class tc_tuning(ctypes.Structure):
    _fields_ = [("light_max_dplus", ctypes.c_int32), ("heavy_block", ctypes.c_int32),
                ("light_block", ctypes.c_int32), ("lds_max_entries", ctypes.c_int32),
                ("algorithm", ctypes.c_int32), ("item_pairs", ctypes.c_int32),
                ("bitmap_words", ctypes.c_int32), ("light_bitmap_pairs", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class tc_fused_tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_st = ctypes.c_int32

_SIGS = {
    "tc_version": (_i32, []),
    "tc_status_string": (ctypes.c_char_p, [_i32]),
    "tc_tuning_default": (_st, [ctypes.POINTER(tc_tuning)]),
    "tc_graph_from_edges": (_st, [_vp, _vp, _i64, _i32, _i32, _vp, ctypes.POINTER(_vp)]),
    "tc_graph_from_csr": (_st, [_vp, _vp, _i32, _i32, _i32, _vp, ctypes.POINTER(_vp)]),
    "tc_batch_create": (_st, [_vp, _vp, _vp, _vp, _i32, _i32, _vp, ctypes.POINTER(_vp)]),
    "tc_fused_tuning_default": (_st, [ctypes.POINTER(tc_fused_tuning)]),
    "tc_batch_fused_workspace_bytes": (_i64, [_i64, _i64, _i32]),
    "tc_batch_fused": (_st, [_vp, _vp, _vp, _vp, _vp, _i32, _i64, _i64, _vp, _vp, _vp, _vp, _vp,
                             _vp, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(tc_fused_tuning), _vp]),
    "tc_batch_fused_noalloc_max_bytes": (_i64, []),
    "tc_batch_fused_noalloc": (_st, [_vp, _vp, _vp, _vp, _vp, _i32, _i64, _i64, _vp, _vp, _vp, _vp,
                                     _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(tc_fused_tuning), _vp]),
    "tc_num_graphs": (_i32, [_vp]),
    "tc_batch_edge_offsets": (_st, [_vp, _vp]),
    "tc_compute": (_st, [_vp, _vp]),
    "tc_compute_tuned": (_st, [_vp, ctypes.POINTER(tc_tuning), _vp]),
    "tc_num_vertices": (_i64, [_vp]),
    "tc_num_edges": (_i64, [_vp]),
    "tc_get_edges": (_st, [_vp, _vp, _vp, _i32, _vp]),
    "tc_get_results": (_st, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "tc_batch_get_results": (_st, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "tc_numerator_algebraic": (_st, [_vp, _vp, _i32, _vp]),
    "tc_trim_memory": (_st, []),
    "tc_edge_text_read": (_st, [ctypes.c_char_p, _vp, _vp, _i64, ctypes.POINTER(_i64),
                                ctypes.POINTER(_i64), _i32]),
    "tc_relabel_ids": (_st, [_vp, _vp, _i64, _vp, _vp, _vp, ctypes.POINTER(_i64), _i32, _vp]),
    "tc_graph_device_bytes": (_st, [_vp, ctypes.POINTER(_i64)]),
    "tc_estimate_device_bytes": (_i64, [_i64, _i32]),
    "tc_compute_bytes": (_st, [_vp, ctypes.POINTER(tc_tuning), _vp, ctypes.POINTER(_i64)]),
    "tc_set_memory_limit": (_st, [_i64]),
    "tc_memory_stats": (_st, [ctypes.POINTER(_i64)] * 4 + [_i32]),
    "tc_graph_destroy": (None, [_vp]),
    "tc_top_k": (_st, [_vp, _i32, _vp, _vp, ctypes.POINTER(_i32), _i32, _vp]),
    "tc_set_profiling": (_st, [_i32]),
    "tc_get_stage_ms": (_st, [_vp, _vp]),
    "tc_get_work_stats": (_st, [_vp, _vp, _vp]),
}

# the last four are launches inside count_light and count_heavy
STAGES = ["csr_build", "degree_rank", "orient", "bin", "count_light", "count_heavy",
          "count_huge", "fold", "tri", "aggregate", "count_light_groups", "count_light_wave",
          "count_light_bitmap", "count_heavy_bitmap16"]
WORK_STATS = ["n", "m", "max_dplus", "rows_light", "rows_heavy", "rows_huge", "cand_light",
              "cand_heavy", "cand_huge", "merge_work", "wedges", "triangles", "edges_light",
              "edges_heavy", "edges_huge", "w_hash", "algorithm", "cand_heavy_16",
              "edges_heavy_16", "rows_heavy_16"]


def load(path=None):
    """Load libtc.so (built in-tree by the package build)."""
    global _lib
    if _lib is None:
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(f"libtc.so not found at {p}: build the HIP library first")
        L = ctypes.CDLL(p)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, where):
    if status < 0:
        raise TCError(status, where)
    return int(status)


# ---------------------------------------------------------------------------
# One-to-one wrappers of the C entry points
# ---------------------------------------------------------------------------
def tc_version():
    return int(load().tc_version())


def tc_status_string(status):
    return load().tc_status_string(int(status)).decode()


def tc_tuning_default():
    t = tc_tuning()
    _check(load().tc_tuning_default(ctypes.byref(t)), "tc_tuning_default")
    return t


def tc_graph_from_edges(src, dst, num_pairs, n, mem_kind, stream):
    h = _vp()
    _check(load().tc_graph_from_edges(src, dst, int(num_pairs), int(n), int(mem_kind), stream,
                                      ctypes.byref(h)), "tc_graph_from_edges")
    return h


def tc_graph_from_csr(row_ptr, col, n, mem_kind, assume_simple_sorted, stream):
    h = _vp()
    _check(load().tc_graph_from_csr(row_ptr, col, int(n), int(mem_kind),
                                    1 if assume_simple_sorted else 0, stream, ctypes.byref(h)),
           "tc_graph_from_csr")
    return h


def tc_batch_create(src, dst, graph_pair_off, graph_vtx_off, num_graphs, mem_kind, stream):
    h = _vp()
    _check(load().tc_batch_create(src, dst, graph_pair_off, graph_vtx_off, int(num_graphs),
                                  int(mem_kind), stream, ctypes.byref(h)), "tc_batch_create")
    return h


def tc_fused_tuning_default():
    t = tc_fused_tuning()
    _check(load().tc_fused_tuning_default(ctypes.byref(t)), "tc_fused_tuning_default")
    return t


def tc_batch_fused_workspace_bytes(num_pairs, num_vertices, num_graphs):
    return int(load().tc_batch_fused_workspace_bytes(int(num_pairs), int(num_vertices),
                                                      int(num_graphs)))


def tc_batch_fused(src, dst, graph_pair_off, graph_vtx_off, order, num_graphs, num_pairs,
                   num_vertices, eu, ev, support, num_edges, tri, triG, num, tc, status, workspace,
                   workspace_bytes, tuning, stream):
    return _check(load().tc_batch_fused(
        src, dst, graph_pair_off, graph_vtx_off, order, int(num_graphs), int(num_pairs),
        int(num_vertices), eu, ev, support, num_edges, tri, triG, num, tc, status, workspace,
        int(workspace_bytes), ctypes.byref(tuning) if tuning is not None else None, stream),
        "tc_batch_fused")


def tc_batch_fused_noalloc_max_bytes():
    return int(load().tc_batch_fused_noalloc_max_bytes())


def tc_batch_fused_noalloc(src, dst, graph_pair_off, graph_vtx_off, order, num_graphs, num_pairs,
                           num_vertices, eu, ev, support, num_edges, tri, triG, num, tc, status,
                           tuning, stream):
    return _check(load().tc_batch_fused_noalloc(
        src, dst, graph_pair_off, graph_vtx_off, order, int(num_graphs), int(num_pairs),
        int(num_vertices), eu, ev, support, num_edges, tri, triG, num, tc, status,
        ctypes.byref(tuning) if tuning is not None else None, stream), "tc_batch_fused_noalloc")


def tc_num_graphs(h):
    return int(load().tc_num_graphs(h))


def tc_batch_edge_offsets(h, edge_off):
    return _check(load().tc_batch_edge_offsets(h, edge_off), "tc_batch_edge_offsets")


def tc_compute(h, stream):
    return _check(load().tc_compute(h, stream), "tc_compute")


def tc_compute_tuned(h, tuning, stream):
    return _check(load().tc_compute_tuned(h, ctypes.byref(tuning) if tuning is not None else None,
                                          stream), "tc_compute_tuned")


def tc_num_vertices(h):
    return int(load().tc_num_vertices(h))


def tc_num_edges(h):
    return int(load().tc_num_edges(h))


def tc_get_edges(h, u, v, mem_kind, stream):
    return _check(load().tc_get_edges(h, u, v, int(mem_kind), stream), "tc_get_edges")


def tc_get_results(h, tri, support, triG, num, tc, mem_kind, stream):
    return _check(load().tc_get_results(h, tri, support, triG, num, tc, int(mem_kind), stream),
                  "tc_get_results")


def tc_batch_get_results(h, tri, support, triG, num, tc, mem_kind, stream):
    return _check(load().tc_batch_get_results(h, tri, support, triG, num, tc, int(mem_kind),
                                              stream), "tc_batch_get_results")


def tc_numerator_algebraic(h, num, mem_kind, stream):
    return _check(load().tc_numerator_algebraic(h, num, int(mem_kind), stream),
                  "tc_numerator_algebraic")


def tc_edge_text_read(path, src=None, dst=None, capacity=0, nthreads=0):
    """(status, num_pairs, bad_line); fills src/dst (int64 arrays) when given."""
    np_ = _i64(0)
    bad = _i64(-1)
    st = load().tc_edge_text_read(os.fsencode(path), _ptr(src), _ptr(dst), int(capacity),
                                  ctypes.byref(np_), ctypes.byref(bad), int(nthreads))
    return int(st), int(np_.value), int(bad.value)


def read_edge_text(path, nthreads=0):
    """Pairs of a text edge list as two int64 arrays (original ids)."""
    st, P, bad = tc_edge_text_read(path, nthreads=nthreads)
    if st == TC_ERR_INVALID_ARG and bad > 0:
        raise TCError(st, f"tc_edge_text_read: {path}: malformed line {bad}")
    _check(st, "tc_edge_text_read")
    src = np.empty(max(P, 1), np.int64)
    dst = np.empty(max(P, 1), np.int64)
    st, P2, bad = tc_edge_text_read(path, src, dst, src.shape[0], nthreads)
    _check(st, "tc_edge_text_read")
    assert P2 == P
    return src[:P], dst[:P]


def tc_relabel_ids(src, dst, num_pairs, src32, dst32, ids, mem_kind, stream):
    n = _i64(0)
    _check(load().tc_relabel_ids(src, dst, int(num_pairs), src32, dst32, ids, ctypes.byref(n),
                                 int(mem_kind), stream), "tc_relabel_ids")
    return int(n.value)


def relabel(src, dst, stream=None):
    """Order-preserving relabel of int64 ids to 0..n-1 on the device.

    Host arrays in, host arrays out: (src32, dst32, ids, n) where ids[k] is
    the original id of new vertex k."""
    src = np.ascontiguousarray(src, np.int64)
    dst = np.ascontiguousarray(dst, np.int64)
    P = src.shape[0]
    s32 = np.empty(max(P, 1), np.int32)
    d32 = np.empty(max(P, 1), np.int32)
    ids = np.empty(max(2 * P, 1), np.int64)
    n = tc_relabel_ids(_ptr(src), _ptr(dst), P, _ptr(s32), _ptr(d32), _ptr(ids), TC_MEM_HOST,
                       stream)
    return s32[:P], d32[:P], ids[:n], n


def tc_graph_device_bytes(h):
    b = _i64(0)
    _check(load().tc_graph_device_bytes(h, ctypes.byref(b)), "tc_graph_device_bytes")
    return int(b.value)


def tc_estimate_device_bytes(num_pairs, n):
    return int(load().tc_estimate_device_bytes(int(num_pairs), int(n)))


def tc_compute_bytes(h, tuning=None, stream=None):
    b = _i64(0)
    t = None
    if tuning is not None:
        t = tuning if isinstance(tuning, tc_tuning) else tuning_from_dict(tuning)
        t = ctypes.byref(t)
    _check(load().tc_compute_bytes(h, t, stream, ctypes.byref(b)), "tc_compute_bytes")
    return int(b.value)


def tc_set_memory_limit(nbytes):
    return _check(load().tc_set_memory_limit(int(nbytes)), "tc_set_memory_limit")


def tc_memory_stats(reset_peaks=False):
    v = [_i64(0) for _ in range(4)]
    _check(load().tc_memory_stats(*[ctypes.byref(x) for x in v], 1 if reset_peaks else 0),
           "tc_memory_stats")
    return dict(zip(("held", "in_use", "peak_held", "peak_in_use"), (int(x.value) for x in v)))


def tc_graph_destroy(h):
    if h:
        load().tc_graph_destroy(h)


def tc_top_k(h, k, vertices, values, mem_kind, stream):
    ko = _i32(0)
    _check(load().tc_top_k(h, int(k), vertices, values, ctypes.byref(ko), int(mem_kind), stream),
           "tc_top_k")
    return int(ko.value)


def tc_trim_memory():
    return _check(load().tc_trim_memory(), "tc_trim_memory")


def tc_set_profiling(on):
    return _check(load().tc_set_profiling(1 if on else 0), "tc_set_profiling")


def tc_get_stage_ms(h):
    ms = (ctypes.c_double * len(STAGES))()
    _check(load().tc_get_stage_ms(h, ctypes.cast(ms, _vp)), "tc_get_stage_ms")
    return dict(zip(STAGES, list(ms)))


def tc_get_work_stats(h, stream):
    st = (ctypes.c_int64 * len(WORK_STATS))()
    _check(load().tc_get_work_stats(h, ctypes.cast(st, _vp), stream), "tc_get_work_stats")
    return dict(zip(WORK_STATS, [int(x) for x in st]))


# ---------------------------------------------------------------------------
# Convenience wrapper
# ---------------------------------------------------------------------------
def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x):
    if x is None:
        return None
    if _is_torch(x):
        return x.data_ptr()
    return x.ctypes.data


def current_stream():
    """hipStream_t of torch's current stream (as an int), or None."""
    import torch
    return torch.cuda.current_stream().cuda_stream


def _streams(stream):
    """(torch's current stream, the handle's stream as a torch stream, or
    None when it is the current one).  Device tensors made on the current
    stream and used by the library on another need both orders: the
    library's work after the current stream's, and the caller's later work
    after the library's."""
    import torch
    cur = torch.cuda.current_stream()
    if stream is None or int(stream) == int(cur.cuda_stream):
        return cur, None
    return cur, torch.cuda.ExternalStream(int(stream))


class Graph:
    """A libtc handle.  Build with ``from_edges`` / ``from_csr`` / ``batch``."""

    def __init__(self, handle, stream=None):
        self.h = handle
        self.stream = stream
        self.status = None

    # -- construction ---------------------------------------------------------
    @classmethod
    def from_edges(cls, src, dst, n, stream=None):
        dev = _is_torch(src) and src.is_cuda
        if dev:
            import torch
            src = src.to(torch.int32).contiguous()
            dst = dst.to(torch.int32).contiguous()
            if stream is None:
                stream = current_stream()
            _, own = _streams(stream)
            if own is not None:  # the pairs (and their conversion) are on the current stream
                own.wait_stream(torch.cuda.current_stream())
        else:
            src = np.ascontiguousarray(src, np.int32)
            dst = np.ascontiguousarray(dst, np.int32)
        h = tc_graph_from_edges(_ptr(src), _ptr(dst), src.shape[0], n,
                                TC_MEM_DEVICE if dev else TC_MEM_HOST, stream)
        return cls(h, stream)

    @classmethod
    def from_csr(cls, row_ptr, col, n, stream=None, assume_simple_sorted=False):
        dev = _is_torch(row_ptr) and row_ptr.is_cuda
        if dev:
            if stream is None:
                stream = current_stream()
            cur, own = _streams(stream)
            if own is not None:
                own.wait_stream(cur)
        else:
            row_ptr = np.ascontiguousarray(row_ptr, np.int64)
            col = np.ascontiguousarray(col, np.int32)
        h = tc_graph_from_csr(_ptr(row_ptr), _ptr(col), n, TC_MEM_DEVICE if dev else TC_MEM_HOST,
                              assume_simple_sorted, stream)
        return cls(h, stream)

    @classmethod
    def from_text(cls, path, stream=None, nthreads=0):
        """Reads a text edge list, relabels its ids to 0..n-1 (order
        preserving) and builds the graph.  Returns (graph, ids) where ids[k]
        is the original id of vertex k."""
        src, dst = read_edge_text(path, nthreads)
        s32, d32, ids, n = relabel(src, dst, stream)
        return cls.from_edges(s32, d32, n, stream=stream), ids

    @classmethod
    def batch(cls, src, dst, pair_off, vtx_off, stream=None):
        dev = _is_torch(src) and src.is_cuda
        if dev and stream is None:
            stream = current_stream()
        if dev:
            cur, own = _streams(stream)
            if own is not None:
                own.wait_stream(cur)
        if not dev:
            src = np.ascontiguousarray(src, np.int32)
            dst = np.ascontiguousarray(dst, np.int32)
        po = np.ascontiguousarray(pair_off, np.int64)
        vo = np.ascontiguousarray(vtx_off, np.int64)
        h = tc_batch_create(_ptr(src), _ptr(dst), po.ctypes.data, vo.ctypes.data, po.shape[0] - 1,
                            TC_MEM_DEVICE if dev else TC_MEM_HOST, stream)
        return cls(h, stream)

    # -- queries ----------------------------------------------------------------
    @property
    def n(self):
        return tc_num_vertices(self.h)

    @property
    def m(self):
        return tc_num_edges(self.h)

    @property
    def num_graphs(self):
        return tc_num_graphs(self.h)

    def device_bytes(self):
        return tc_graph_device_bytes(self.h)

    def compute_bytes(self, tuning=None):
        """Upper bound of the device bytes compute(tuning) adds (waits for
        the handle's stream)."""
        return tc_compute_bytes(self.h, tuning, self.stream)

    def compute(self, tuning=None):
        if tuning is None:
            self.status = tc_compute(self.h, self.stream)
        else:
            t = tuning if isinstance(tuning, tc_tuning) else tuning_from_dict(tuning)
            self.status = tc_compute_tuned(self.h, t, self.stream)
        return self.status

    def edges(self):
        m = self.m
        u = np.empty(max(m, 1), np.int32)
        v = np.empty(max(m, 1), np.int32)
        tc_get_edges(self.h, _ptr(u), _ptr(v), TC_MEM_HOST, self.stream)
        return u[:m], v[:m]

    def edge_offsets(self):
        off = np.empty(self.num_graphs + 1, np.int64)
        tc_batch_edge_offsets(self.h, _ptr(off))
        return off

    def results(self):
        """Host copies: dict(tri, support, triG, num, tc)."""
        n, m, G = self.n, self.m, self.num_graphs
        out = {
            "tri": np.empty(max(n, 1), np.uint64),
            "support": np.empty(max(m, 1), np.uint64),
            "triG": np.empty(G, np.uint64),
            "num": np.empty(max(n, 1), np.uint64),
            "tc": np.empty(max(n, 1), np.float64),
        }
        tc_get_results(self.h, _ptr(out["tri"]), _ptr(out["support"]), _ptr(out["triG"]),
                       _ptr(out["num"]), _ptr(out["tc"]), TC_MEM_HOST, self.stream)
        out["tri"] = out["tri"][:n]
        out["support"] = out["support"][:m]
        out["num"] = out["num"][:n]
        out["tc"] = out["tc"][:n]
        return out

    def results_device(self):
        """Device copies as torch tensors (int64 views of the uint64 data),
        ready for use on the caller's current stream.

        The library copies on the handle's stream.  When that is not the
        current stream, the handle's stream first waits for the current one
        (the new tensors' memory may still be in use there) and the current
        stream then waits for the copies."""
        import torch
        n, m, G = self.n, self.m, self.num_graphs
        dev = torch.device("cuda")
        cur, own = _streams(self.stream)
        out = {
            "tri": torch.empty(max(n, 1), dtype=torch.int64, device=dev),
            "support": torch.empty(max(m, 1), dtype=torch.int64, device=dev),
            "triG": torch.empty(G, dtype=torch.int64, device=dev),
            "num": torch.empty(max(n, 1), dtype=torch.int64, device=dev),
            "tc": torch.empty(max(n, 1), dtype=torch.float64, device=dev),
        }
        if own is not None:
            own.wait_stream(cur)
        tc_get_results(self.h, _ptr(out["tri"]), _ptr(out["support"]), _ptr(out["triG"]),
                       _ptr(out["num"]), _ptr(out["tc"]), TC_MEM_DEVICE, self.stream)
        if own is not None:
            cur.wait_stream(own)
        return out

    def numerator_algebraic(self):
        """num[] by Algorithm 3's algebraic form (host copy)."""
        n = self.n
        out = np.empty(max(n, 1), np.uint64)
        tc_numerator_algebraic(self.h, _ptr(out), TC_MEM_HOST, self.stream)
        return out[:n]

    def stage_ms(self):
        return tc_get_stage_ms(self.h)

    def work_stats(self):
        return tc_get_work_stats(self.h, self.stream)

    def top_k(self, k):
        k = min(int(k), self.n)
        verts = np.empty(max(k, 1), np.int32)
        vals = np.empty(max(k, 1), np.float64)
        got = tc_top_k(self.h, k, _ptr(verts), _ptr(vals), TC_MEM_HOST, self.stream)
        return verts[:got], vals[:got]

    def close(self):
        if self.h:
            tc_graph_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FusedBatch:
    """Device buffers for ``tc_batch_fused`` over one batch layout.

    ``src``/``dst`` are device int32 tensors of local ids; ``pair_off`` and
    ``vtx_off`` host arrays of G+1 offsets.  ``order`` is "largest_first"
    (graphs taken by pair count, largest first), None (index order) or an
    explicit permutation.  ``run()`` queues the one launch (plus the queue
    reset) on ``stream`` and allocates nothing, so it can be captured in a
    CUDA/HIP graph.  Outputs stay on the device in the attributes named like
    the C arguments (uint64 data in int64 tensors).
    """

    def __init__(self, src, dst, pair_off, vtx_off, order="largest_first", tuning=None,
                 stream=None):
        import torch
        dev = src.device
        po = np.ascontiguousarray(pair_off, np.int64)
        vo = np.ascontiguousarray(vtx_off, np.int64)
        self.G = int(po.shape[0] - 1)
        self.P = int(po[-1])
        self.N = int(vo[-1])
        self.h_pair_off, self.h_vtx_off = po, vo
        self.src = src.to(torch.int32).contiguous()
        self.dst = dst.to(torch.int32).contiguous()
        self.pair_off = torch.from_numpy(po).to(dev)
        self.vtx_off = torch.from_numpy(vo).to(dev)
        if isinstance(order, str) and order == "largest_first":
            order = np.argsort(-np.diff(po), kind="stable").astype(np.int32)
        self.order = None if order is None else torch.from_numpy(
            np.ascontiguousarray(order, np.int32)).to(dev)
        if tuning is None or isinstance(tuning, tc_fused_tuning):
            self.tuning = tuning
        else:
            self.tuning = tc_fused_tuning_default()
            for k, v in tuning.items():
                setattr(self.tuning, k, int(v))
        self.stream = stream if stream is not None else current_stream()
        P1, N1, G1 = max(self.P, 1), max(self.N, 1), max(self.G, 1)
        self.eu = torch.empty(P1, dtype=torch.int32, device=dev)
        self.ev = torch.empty(P1, dtype=torch.int32, device=dev)
        self.support = torch.empty(P1, dtype=torch.int64, device=dev)
        self.num_edges = torch.empty(G1, dtype=torch.int64, device=dev)
        self.tri = torch.empty(N1, dtype=torch.int64, device=dev)
        self.num = torch.empty(N1, dtype=torch.int64, device=dev)
        self.tc = torch.empty(N1, dtype=torch.float64, device=dev)
        self.triG = torch.empty(G1, dtype=torch.int64, device=dev)
        self.status = torch.empty(G1, dtype=torch.int32, device=dev)
        self.ws_bytes = tc_batch_fused_workspace_bytes(self.P, self.N, self.G)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self.ws_ptr = self.workspace.data_ptr() + off

    def run(self):
        """One launch on ``stream``.  When that is not torch's current
        stream, the launch waits for the current stream (where the buffers
        were made) and the current stream waits for the launch."""
        cur, own = _streams(self.stream)
        if own is not None:
            own.wait_stream(cur)
        st = self._launch()
        if own is not None:
            cur.wait_stream(own)
        return st

    def _launch(self):
        return tc_batch_fused(
            _ptr(self.src), _ptr(self.dst), _ptr(self.pair_off), _ptr(self.vtx_off),
            _ptr(self.order), self.G, self.P, self.N, _ptr(self.eu), _ptr(self.ev),
            _ptr(self.support), _ptr(self.num_edges), _ptr(self.tri), _ptr(self.triG),
            _ptr(self.num), _ptr(self.tc), _ptr(self.status), self.ws_ptr, self.ws_bytes,
            self.tuning, self.stream)

    def results(self):
        """Host copies: dict(eu, ev, support, num_edges, tri, triG, num, tc, status)
        with the C layout (edges at the pair offsets)."""
        P, N, G = self.P, self.N, self.G
        cur, own = _streams(self.stream)
        if own is not None:  # the copies below run on the current stream
            cur.wait_stream(own)
        out = {"eu": self.eu[:P], "ev": self.ev[:P], "support": self.support[:P],
               "num_edges": self.num_edges[:G], "tri": self.tri[:N], "triG": self.triG[:G],
               "num": self.num[:N], "tc": self.tc[:N], "status": self.status[:G]}
        out = {k: v.cpu().numpy() for k, v in out.items()}
        for k in ("support", "tri", "triG", "num"):
            out[k] = out[k].view(np.uint64)
        return out

    def graph(self, res, g):
        """Graph g's slice of host results: eu, ev, support (m_g entries),
        tri, num, tc (n_g entries), triG, status."""
        pa, va, vb = int(self.h_pair_off[g]), int(self.h_vtx_off[g]), int(self.h_vtx_off[g + 1])
        m = int(res["num_edges"][g])
        return {"eu": res["eu"][pa:pa + m], "ev": res["ev"][pa:pa + m],
                "support": res["support"][pa:pa + m], "tri": res["tri"][va:vb],
                "num": res["num"][va:vb], "tc": res["tc"][va:vb],
                "triG": res["triG"][g:g + 1], "status": int(res["status"][g])}


def tuning_from_dict(d):
    t = tc_tuning_default()
    for k, v in d.items():
        setattr(t, k, int(v))
    return t
