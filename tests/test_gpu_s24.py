"""GPU parity at the benchmark's full size: R-MAT scale 24 (2^28 pairs,
m = 260.4 M) with the stored tuning that bench.py times.

Every output of the HIP path is compared with a full run of the oracle O2
(the appendix's Procedure 2 with counts, then Algorithm 2, on the host's
threads) on the same pairs: the canonical edge list, every edge's support,
every vertex's triangle count, △(G), every numerator and the bit pattern of
every TC value.  The three largest hubs' triangle counts are also checked
by the definition (common neighbours by marking), a formulation that shares
nothing with O2's orientation.
"""
import time

import numpy as np
import pytest

from oracle import native
from paper_2105_00110_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.timeout(1200)
def test_rmat_s24_full_parity_at_bench_configuration(tclib):
    from paper_2105_00110_amd import autotune
    src, dst, n = gg.rmat(24, 16, seed=24)
    tuning = autotune.load("rmat_s24_ef16")
    _say("R-MAT s24 gpu, tuning", tuning)
    g = tclib.Graph.from_edges(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(), n)
    st = g.compute(tuning)
    r = g.results()
    eu, ev = g.edges()
    g.close()
    torch.cuda.empty_cache()
    tclib.tc_trim_memory()
    triG = int(r["triG"][0])
    assert st == 0 and triG > 0
    threads = native.host_threads()
    _say("oracle O2 on", threads, "threads")
    t0 = time.perf_counter()
    ref = native.o2_paper(src, dst, n, nthreads=threads)
    _say(f"oracle O2 done in {time.perf_counter() - t0:.1f} s, m = {ref.m}, triG = {ref.triG}")
    assert ref.status == st
    assert eu.shape[0] == ref.m
    np.testing.assert_array_equal(eu, ref.eu)
    np.testing.assert_array_equal(ev, ref.ev)
    np.testing.assert_array_equal(r["support"], ref.sup)
    np.testing.assert_array_equal(r["tri"], ref.tri)
    assert triG == ref.triG
    np.testing.assert_array_equal(r["num"], ref.num)
    np.testing.assert_array_equal(r["tc"].view(np.uint64), ref.tc.view(np.uint64))
    # properties that hold at any size, on the oracle's own outputs
    assert int(ref.tri.sum()) == 3 * ref.triG == int(ref.sup.sum())
    assert np.all(ref.num <= np.uint64(3 * ref.triG))
    del ref
    # the largest hubs by the definition, independently of O2
    deg = np.bincount(eu, minlength=n) + np.bincount(ev, minlength=n)
    hubs = np.argsort(deg)[-3:].astype(np.int32)
    _say("definition point queries on the hubs", hubs.tolist(), deg[hubs].tolist())
    q = native.PointQuery(src, dst, n)
    np.testing.assert_array_equal(q.tri(hubs), r["tri"][hubs])
    q.close()
