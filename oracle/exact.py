"""Exact rational triangle centrality -- test infrastructure.

``tc_fraction`` is Definition 1 evaluated in exact rational arithmetic from
tri and the triangle-neighbour sets, with the 1/3 weight on the closed
triangle neighbourhood N△[v] exactly as printed.  ``correctly_rounded``
turns a Fraction into the nearest float64 (Python rounds Fraction -> float
correctly), which is what a single IEEE division of two exactly
representable integers also yields.
"""
from fractions import Fraction


def tc_fraction(v, adj, tri, core, triG):
    """Definition 1 for vertex v.

    adj[v]: neighbour set; tri[u]: triangle count; core[v]: N△(v);
    triG: triangles in the graph (must be > 0).
    """
    closed = set(core[v]) | {v}
    first = Fraction(sum(int(tri[u]) for u in closed), 3)
    second = Fraction(sum(int(tri[w]) for w in adj[v] if w not in core[v]))
    return (first + second) / int(triG)


def correctly_rounded(fr):
    return float(fr)
