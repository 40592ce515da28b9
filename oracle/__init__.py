"""CPU oracle for triangle centrality -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library (``paper_2105_00110_amd``) and never imports it; both sides only
share the seeded input generators.

Implementations (all return the same exact integers and the same float64
quotient; see each module for the passage it follows):

* ``brute``      -- O0: enumeration of all vertex triples (tiny graphs).
* ``algebraic``  -- O3: Proposition 2, dense matrices in float64.
* ``native``     -- O1 (definition, per-edge common neighbours) and
                    O2 (Procedure 2 + Algorithm 2 of the paper), in C.
* ``exact``      -- the same quotient as an exact rational, for pins.

Parity status: every function here is pinned by the ``-m "not gpu"``
tests (closed forms of the paper's Observations, its worked example and
figure graphs, brute force on tiny inputs, and cross-formulation
agreement); none is "parity unpinned".
"""
from .result import OracleResult  # noqa: F401
