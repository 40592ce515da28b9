"""O0: brute-force triangle centrality on tiny graphs -- test infrastructure.

Plain Python over all vertex triples i < j < k: a triple whose three pairs
are edges is a triangle.  Every triangle adds one to tri of its three
vertices, one to the support of its three edges and one to triG.  Then
N△(v) = {u ∈ N(v) : sup(u,v) > 0} (Sec. "Notation") and Definition 1's
numerator times 3·triG,
    num(v) = tri(v) + Σ_{u ∈ N△(v)} tri(u) + 3 Σ_{w ∈ N(v)\\N△(v)} tri(w),
and tc(v) = num(v) / (3·triG) as one float64 division.
O(n^3): meant for n up to a couple of hundred.
"""
from itertools import combinations

import numpy as np

from .result import OracleResult


def normalise_pairs(src, dst, n):
    """Simple undirected graph: self-loops dropped, duplicates merged."""
    edges = set()
    for a, b in zip(list(map(int, src)), list(map(int, dst))):
        if not (0 <= a < n and 0 <= b < n):
            raise ValueError("vertex id out of range")
        if a != b:
            edges.add((min(a, b), max(a, b)))
    return sorted(edges)


def brute_force(src, dst, n):
    n = int(n)
    edges = normalise_pairs(src, dst, n)
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    tri = [0] * n
    sup = {e: 0 for e in edges}
    triG = 0
    for i, j, k in combinations(range(n), 3):
        if j in adj[i] and k in adj[i] and k in adj[j]:
            triG += 1
            for v in (i, j, k):
                tri[v] += 1
            for e in ((i, j), (i, k), (j, k)):
                sup[e] += 1
    num = [0] * n
    for v in range(n):
        acc = tri[v]
        for u in adj[v]:
            in_core = sup[(min(u, v), max(u, v))] > 0
            acc += tri[u] if in_core else 3 * tri[u]
        num[v] = acc
    tc = [0.0 if triG == 0 else float(num[v]) / float(3 * triG) for v in range(n)]
    eu = np.array([e[0] for e in edges], dtype=np.int32)
    ev = np.array([e[1] for e in edges], dtype=np.int32)
    return OracleResult(n=n, eu=eu, ev=ev,
                        sup=np.array([sup[e] for e in edges], dtype=np.uint64),
                        tri=np.array(tri, dtype=np.uint64), triG=triG,
                        num=np.array(num, dtype=np.uint64),
                        tc=np.array(tc, dtype=np.float64), status=0 if triG else 1)
