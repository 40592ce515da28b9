"""O3: Proposition 2 with dense matrices -- test infrastructure.

Proposition 2 (Sec. "Algebraic Form") and Algorithm 3: with the adjacency
matrix A and the graph triangle matrix T = A^2 ∘ A,
    tc = (3A - 2·bin(T) + I) · T·1 / (1ᵀ T 1).
In float64 with integer entries below 2^53 every product here is exact.
The quoted theorem gives tri = (T·1)/2 and triG = (1ᵀT1)/6, so
    num = 3·triG·tc = (3A - 2·bin(T) + I) · (T·1) / 2,
which is returned as an integer; ``tc`` is then num / (3·triG) as one
division (the same rounding as every other implementation), and
``tc_direct`` is Algorithm 3's own last line X·y / k, for comparison only.
"""
import numpy as np

from .brute import normalise_pairs
from .result import OracleResult


def algebraic(src, dst, n):
    n = int(n)
    edges = normalise_pairs(src, dst, n)
    A = np.zeros((n, n), dtype=np.float64)
    for a, b in edges:
        A[a, b] = A[b, a] = 1.0
    T = (A @ A) * A
    Tb = (T > 0).astype(np.float64)
    X = 3.0 * A - 2.0 * Tb + np.eye(n)
    y = T @ np.ones(n)
    k = float(np.ones(n) @ y)
    numx2 = X @ y
    if not np.all(np.mod(numx2, 2.0) == 0.0) or k % 6.0 != 0.0:
        raise AssertionError("Proposition 2 produced non-integral counts")
    num = (numx2 / 2.0).astype(np.uint64)
    tri = (y / 2.0).astype(np.uint64)
    triG = int(k // 6)
    tc = np.zeros(n) if triG == 0 else num.astype(np.float64) / float(3 * triG)
    eu = np.array([e[0] for e in edges], dtype=np.int32)
    ev = np.array([e[1] for e in edges], dtype=np.int32)
    sup = np.array([T[a, b] for a, b in edges], dtype=np.uint64)
    res = OracleResult(n=n, eu=eu, ev=ev, sup=sup, tri=tri, triG=triG, num=num, tc=tc,
                       status=0 if triG else 1)
    res.tc_direct = np.zeros(n) if k == 0 else numx2 / k
    return res
