"""Seeded synthetic graph workloads (inputs only; no triangle arithmetic).

Every generator returns raw undirected pairs ``(src, dst)`` as int32 numpy
arrays plus the vertex count ``n``.  Pairs may contain self-loops and
duplicates; both the HIP library and the CPU oracle normalise them.  This
module is the only code the two sides share.

Workload recipes (sizes as in the benchmark configurations):

* ``er(n, p, seed)``          Erdős–Rényi G(n, p).
* ``rmat(scale, ef, ...)``    R-MAT, 2^scale vertices, ef·2^scale pairs,
                              (a,b,c,d) = (0.57,0.19,0.19,0.05), no noise,
                              vertex ids scrambled by a keyed bijection.
* ``ba(n, m_attach, ...)``    Barabási–Albert from K_{m+1} plus planted
                              cliques covering ≥ ``cover`` of the vertices.
* ``batched_ba(...)``         the batched workload: many BA graphs.
* small closed-form families (cliques, chains, rings...) for the paper's
  Observations.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "gen", "libtcgen.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")

RMAT_ABC = (0.57, 0.19, 0.19)


def _gen_lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import _build
            _build.build_gen()
        L = ctypes.CDLL(_LIB_PATH)
        L.tcgen_rmat.argtypes = [_i32p, _i32p, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_int]
        L.tcgen_rmat.restype = ctypes.c_int
        L.tcgen_er.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_double, ctypes.c_uint64]
        L.tcgen_er.restype = ctypes.c_int64
        L.tcgen_ba.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_uint64]
        L.tcgen_ba.restype = ctypes.c_int64
        L.tcgen_ba_batch.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_double,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int,
                                     _i64p, _i64p, _i32p, _i32p, ctypes.c_int]
        L.tcgen_ba_batch.restype = ctypes.c_int
        L.tcgen_uniform.argtypes = [_f64p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64]
        L.tcgen_uniform.restype = None
        L.tcgen_write_text.argtypes = [ctypes.c_char_p, _i64p, _i64p, ctypes.c_int64]
        L.tcgen_write_text.restype = ctypes.c_int
        _lib = L
    return _lib


def _threads(nthreads):
    if nthreads:
        return int(nthreads)
    return max(1, min(16, os.cpu_count() or 1))


# ---------------------------------------------------------------------------
# Random families
# ---------------------------------------------------------------------------
def rmat(scale, edge_factor=16, seed=1, abc=RMAT_ABC, scramble=True, nthreads=None,
         num_pairs=None):
    """R-MAT pairs: ``edge_factor · 2^scale`` pairs (or ``num_pairs``)."""
    P = int(num_pairs) if num_pairs is not None else int(edge_factor) << int(scale)
    src = np.empty(P, np.int32)
    dst = np.empty(P, np.int32)
    a, b, c = abc
    st = _gen_lib().tcgen_rmat(src, dst, P, int(scale), a, b, c, int(seed) & (2**64 - 1),
                               1 if scramble else 0, _threads(nthreads))
    if st != 0:
        raise ValueError("bad R-MAT parameters")
    return src, dst, 1 << int(scale)


def er(n, p, seed=1):
    """Erdős–Rényi G(n, p) pairs."""
    L = _gen_lib()
    cnt = L.tcgen_er(None, None, 0, int(n), float(p), int(seed))
    if cnt < 0:
        raise ValueError("bad ER parameters")
    src = np.empty(max(cnt, 1), np.int32)
    dst = np.empty(max(cnt, 1), np.int32)
    got = L.tcgen_er(src.ctypes.data, dst.ctypes.data, max(cnt, 1), int(n), float(p), int(seed))
    assert got == cnt
    return src[:cnt], dst[:cnt], int(n)


def ba(n, m_attach, seed=1, cover=0.10, kmin=5, kmax=20):
    """Barabási–Albert pairs with planted cliques (sizes U{kmin..kmax})."""
    L = _gen_lib()
    args = (int(n), int(m_attach), float(cover), int(kmin), int(kmax), int(seed))
    cnt = L.tcgen_ba(None, None, 0, *args)
    if cnt < 0:
        raise ValueError("bad BA parameters")
    src = np.empty(max(cnt, 1), np.int32)
    dst = np.empty(max(cnt, 1), np.int32)
    got = L.tcgen_ba(src.ctypes.data, dst.ctypes.data, max(cnt, 1), *args)
    assert got == cnt
    return src[:cnt], dst[:cnt], int(n)


def write_text(path, src, dst):
    """Writes int64 pairs as a text edge list ("u v" per line, one '#'
    header line)."""
    src = np.ascontiguousarray(src, np.int64)
    dst = np.ascontiguousarray(dst, np.int64)
    if _gen_lib().tcgen_write_text(os.fsencode(path), src, dst, src.shape[0]) != 0:
        raise OSError(f"cannot write {path}")


def sparse_ids(ids, seed=1):
    """An order-preserving injective map of ids 0..N-1 onto sparse 64-bit
    ids: id -> id * 1000003 + offset + U{0..999} (the gaps make the ids
    non-contiguous; the map stays increasing)."""
    ids = np.asarray(ids, np.int64)
    jitter = np.floor(uniform(int(ids.max()) + 1 if ids.size else 1, seed, 0x1D) * 1000)
    return ids * 1000003 + (1 << 40) + jitter.astype(np.int64)[ids]


def uniform(count, seed, salt):
    out = np.empty(max(int(count), 1), np.float64)
    _gen_lib().tcgen_uniform(out, int(count), int(seed), int(salt))
    return out[:int(count)]


def batched_ba_sizes(num_graphs=4096, seed=4096, n_lo=50, n_hi=20000, m_lo=2, m_hi=16):
    """Per-graph (n, m_attach): n log-uniform in [n_lo, n_hi] rounded to an
    integer, m_attach uniform in {m_lo..m_hi}."""
    u = uniform(num_graphs, seed, 0x4E)
    w = uniform(num_graphs, seed, 0x4D)
    ns = np.rint(np.exp(math.log(n_lo) + u * (math.log(n_hi) - math.log(n_lo)))).astype(np.int32)
    ms = (m_lo + np.floor(w * (m_hi - m_lo + 1))).astype(np.int32)
    ms = np.minimum(ms, m_hi).astype(np.int32)
    return ns, ms


def batched_ba(num_graphs=4096, seed=4096, cover=0.10, kmin=5, kmax=20, ns=None, ms=None,
               nthreads=None):
    """Concatenated BA graphs.

    Returns ``(src, dst, pair_off, vtx_off)``: graph g's pairs are
    ``src/dst[pair_off[g]:pair_off[g+1]]`` with ids local to the graph, and
    its vertices are global ids ``vtx_off[g] .. vtx_off[g+1]-1`` once offset.
    The pairs returned here are LOCAL ids; ``to_global`` adds the offsets.
    """
    if ns is None or ms is None:
        ns, ms = batched_ba_sizes(num_graphs, seed)
    ns = np.ascontiguousarray(ns, np.int32)
    ms = np.ascontiguousarray(ms, np.int32)
    G = ns.shape[0]
    L = _gen_lib()
    counts = np.zeros(G, np.int64)
    dummy_off = np.zeros(G + 1, np.int64)
    d32 = np.zeros(1, np.int32)
    st = L.tcgen_ba_batch(G, ns, ms, float(cover), int(kmin), int(kmax), int(seed), 1, counts,
                          dummy_off, d32, d32, _threads(nthreads))
    if st != 0:
        raise ValueError("bad batched BA parameters")
    pair_off = np.zeros(G + 1, np.int64)
    np.cumsum(counts, out=pair_off[1:])
    P = int(pair_off[-1])
    src = np.empty(max(P, 1), np.int32)
    dst = np.empty(max(P, 1), np.int32)
    st = L.tcgen_ba_batch(G, ns, ms, float(cover), int(kmin), int(kmax), int(seed), 0, counts,
                          pair_off, src, dst, _threads(nthreads))
    if st != 0:
        raise RuntimeError("batched BA generation failed")
    vtx_off = np.zeros(G + 1, np.int64)
    np.cumsum(ns.astype(np.int64), out=vtx_off[1:])
    return src[:P], dst[:P], pair_off, vtx_off


def to_global(src, dst, pair_off, vtx_off):
    """Offset local ids by each graph's first global vertex id."""
    counts = np.diff(pair_off)
    shift = np.repeat(vtx_off[:-1], counts)
    return (src.astype(np.int64) + shift).astype(np.int32), (dst.astype(np.int64) + shift).astype(np.int32)


# ---------------------------------------------------------------------------
# Small structured families (the paper's Observations and figures)
# ---------------------------------------------------------------------------
def _pairs(edges, n):
    if len(edges) == 0:
        return np.zeros(0, np.int32), np.zeros(0, np.int32), int(n)
    a = np.array(edges, dtype=np.int32)
    return a[:, 0].copy(), a[:, 1].copy(), int(n)


def _clique_edges(verts):
    return [(verts[i], verts[j]) for i in range(len(verts)) for j in range(i + 1, len(verts))]


def clique(n):
    """K_n."""
    return _pairs(_clique_edges(list(range(n))), n)


def disjoint_cliques(p, k):
    """p disjoint copies of K_k; copy i holds vertices i*k .. i*k+k-1."""
    edges = []
    for i in range(p):
        edges += _clique_edges(list(range(i * k, i * k + k)))
    return _pairs(edges, p * k)


def bridge_cliques(d, k):
    """Vertex 0 joined to one vertex of each of d disjoint K_k copies
    (vertex 0 is in no triangle)."""
    edges = []
    for i in range(d):
        base = 1 + i * k
        edges += _clique_edges(list(range(base, base + k)))
        edges.append((0, base))
    return _pairs(edges, 1 + d * k)


def clique_chain(p, k, ring=False):
    """p copies of K_k, consecutive copies sharing one vertex; with
    ``ring`` the last copy also shares a vertex with the first.

    Returns ``(src, dst, n, joins, copies)`` where ``joins`` lists the
    shared vertices and ``copies[i]`` the vertex list of copy i.
    """
    copies = []
    nxt = 0
    first = None
    prev_join = None
    for i in range(p):
        verts = []
        if prev_join is not None:
            verts.append(prev_join)
        need = k - len(verts)
        if ring and i == p - 1:
            need -= 1
        verts += list(range(nxt, nxt + need))
        nxt += need
        if ring and i == p - 1:
            verts.append(first)
        if first is None:
            first = verts[0]
        copies.append(verts)
        prev_join = verts[-1] if not (ring and i == p - 1) else None
    joins = set()
    for i in range(p - 1):
        joins |= set(copies[i]) & set(copies[i + 1])
    if ring:
        joins |= set(copies[-1]) & set(copies[0])
    edges = []
    for c in copies:
        edges += _clique_edges(c)
    src, dst, n = _pairs(edges, nxt)
    return src, dst, n, sorted(joins), copies


def single_triangle_with_pendants(pendants=(2, 3, 1)):
    """One triangle {0,1,2}; triangle vertex i also gets pendants[i]
    private neighbours of degree one."""
    edges = [(0, 1), (0, 2), (1, 2)]
    nxt = 3
    for i, c in enumerate(pendants):
        for _ in range(c):
            edges.append((i, nxt))
            nxt += 1
    return _pairs(edges, nxt)


def fig1b_four_k6_hub():
    """Four K6 copies, each with one vertex joined to a hub "a" (vertex 0)."""
    return bridge_cliques(4, 6)
