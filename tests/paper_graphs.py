"""Edge lists drawn in the paper's figures, parsed from its LaTeX source at
test time (never stored in this repository).  Only available where the
paper's source is mounted; tests using it skip elsewhere."""
import os
import re

import numpy as np

PAPER = "/root/reference/PAPER.md"

_DRAW = re.compile(r"\\draw\s*\[edge\]\s*\((\w+)\)\s*--\s*\((\w+)\)\s*;")


def available():
    return os.path.exists(PAPER)


def _figure_block(label):
    with open(PAPER) as f:
        text = f.read()
    end = text.index("\\label{" + label + "}")
    start = text.rfind("\\begin{figure}", 0, end)
    return text[start:end]


def figure_edges(label):
    """Undirected edges of a figure whose TikZ uses ``\\draw [edge] (x) -- (y);``.
    Returns (src, dst, n, names) with vertices numbered in order of first
    appearance in sorted-name order."""
    block = _figure_block(label)
    pairs = _DRAW.findall(block)
    names = sorted({x for p in pairs for x in p}, key=lambda s: (len(s), s))
    idx = {s: i for i, s in enumerate(names)}
    a = np.array([(idx[x], idx[y]) for x, y in pairs], dtype=np.int32)
    return a[:, 0].copy(), a[:, 1].copy(), len(names), names
