"""Result record shared by the oracle implementations (test infrastructure)."""
from dataclasses import dataclass

import numpy as np


@dataclass
class OracleResult:
    """Triangle-centrality outputs for one normalised simple graph.

    ``eu``/``ev``: canonical edges (eu < ev), lexicographic order.
    ``sup``: triangles on each canonical edge (the non-zeros of T = A^2 ∘ A).
    ``tri``: triangles at each vertex; ``triG``: triangles in the graph.
    ``num``: Definition 1's numerator times 3·triG (an integer).
    ``tc``: ``num / (3·triG)`` as one float64 division, 0 when triG == 0.
    ``status``: 0 ok, 1 triangle-free.
    """

    n: int
    eu: np.ndarray
    ev: np.ndarray
    sup: np.ndarray
    tri: np.ndarray
    triG: int
    num: np.ndarray
    tc: np.ndarray
    status: int = 0

    @property
    def m(self) -> int:
        return int(self.eu.shape[0])
