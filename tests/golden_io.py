"""Reader for the small text fixtures under tests/golden/."""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    n = None
    edges = []
    facts = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "n":
                n = int(tok[1])
            elif tok[0] == "e":
                edges.append((int(tok[1]), int(tok[2])))
            else:
                vals = []
                for t in tok[1:]:
                    vals.append(Fraction(t) if "/" in t else int(t))
                facts.setdefault(tok[0], []).append(vals)
    if edges:
        a = np.array(edges, dtype=np.int32)
        src, dst = a[:, 0].copy(), a[:, 1].copy()
    else:
        src = dst = np.zeros(0, np.int32)
    return src, dst, n, facts
