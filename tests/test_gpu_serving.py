"""GPU: the batched configuration, the serving loop and the autotuner.

* 4096 Barabasi-Albert graphs with planted cliques as one batch: sampled
  graphs bit-exact against the oracle, every graph's invariants, and the
  whole batch equal to one graph per launch on a prefix of the graphs.
* Serving: every reply of a mixed, overlapping, batched run equals the same
  request run alone (bit for bit), and sampled replies equal the oracle;
  graphs kept resident answer later top-k and vertex queries, also under a
  budget tight enough to evict them.
* Autotuner: a short search leaves every result unchanged.
"""
import numpy as np
import pytest

from oracle import native
from paper_2105_00110_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


def _check_oracle(res, ref):
    np.testing.assert_array_equal(res["support"], ref.sup)
    np.testing.assert_array_equal(res["tri"], ref.tri)
    assert int(res["triG"][0]) == ref.triG
    np.testing.assert_array_equal(res["num"], ref.num)
    np.testing.assert_array_equal(res["tc"].view(np.uint64), ref.tc.view(np.uint64))


@pytest.fixture(scope="module")
def batch4096():
    return gg.batched_ba(4096, seed=4096)


def test_batched_4096_sampled_oracle_and_invariants(tclib, batch4096):
    src, dst, po, vo = batch4096
    G = len(po) - 1
    _say("batched BA", G, "graphs", len(src), "pairs")
    ds, dd = torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda()
    g = tclib.Graph.batch(ds, dd, po, vo)
    g.compute()
    res = g.results()
    eoff = g.edge_offsets()
    eu, ev = g.edges()
    g.close()
    tri, sup, triG, num, tcv = res["tri"], res["support"], res["triG"], res["num"], res["tc"]
    assert len(triG) == G and eoff[0] == 0 and eoff[-1] == len(sup)
    # per-graph invariants over every graph: sum tri = 3 triG, sum sup = 3 triG,
    # 0 <= num <= 3 triG, 0 <= tc <= 1, edges stay inside their graph
    tri_sum = np.add.reduceat(tri, vo[:-1].astype(np.int64)) if len(tri) else tri
    sizes = np.diff(vo)
    assert np.all(sizes > 0)
    np.testing.assert_array_equal(tri_sum, 3 * triG)
    sup_sum = np.array([int(sup[eoff[i]:eoff[i + 1]].sum()) for i in range(G)], np.uint64)
    np.testing.assert_array_equal(sup_sum, 3 * triG)
    owner = np.repeat(np.arange(G), sizes)
    np.testing.assert_array_equal(owner[eu], owner[ev])
    assert np.all(num <= 3 * triG[owner])
    assert np.all((tcv >= 0) & (tcv <= 1))
    # sampled graphs against the oracle: smallest, largest, densest and a spread
    m_per = np.diff(eoff)
    pick = {int(np.argmin(sizes)), int(np.argmax(sizes)), int(np.argmax(m_per / sizes))}
    pick |= set(range(0, G, 512))
    for gi in sorted(pick):
        _say("oracle graph", gi, "n", int(sizes[gi]), "m", int(m_per[gi]))
        a, b = int(po[gi]), int(po[gi + 1])
        ref = native.o2_paper(src[a:b], dst[a:b], int(sizes[gi]))
        va, vb = int(vo[gi]), int(vo[gi + 1])
        ea, eb = int(eoff[gi]), int(eoff[gi + 1])
        one = {"support": sup[ea:eb], "tri": tri[va:vb], "triG": triG[gi:gi + 1],
               "num": num[va:vb], "tc": tcv[va:vb]}
        _check_oracle(one, ref)
        np.testing.assert_array_equal(eu[ea:eb] - va, ref.eu)
        np.testing.assert_array_equal(ev[ea:eb] - va, ref.ev)


def test_batched_prefix_equals_one_graph_per_launch(tclib, batch4096):
    src, dst, po, vo = batch4096
    G = 256
    P = int(po[G])
    ds, dd = torch.from_numpy(src[:P]).cuda(), torch.from_numpy(dst[:P]).cuda()
    _say("batch prefix", G, "graphs vs one graph per launch")
    g = tclib.Graph.batch(ds, dd, po[:G + 1], vo[:G + 1])
    g.compute()
    res = g.results()
    eoff = g.edge_offsets()
    g.close()
    for gi in range(G):
        a, b = int(po[gi]), int(po[gi + 1])
        h = tclib.Graph.from_edges(ds[a:b], dd[a:b], int(vo[gi + 1] - vo[gi]))
        h.compute()
        r1 = h.results()
        h.close()
        va, vb = int(vo[gi]), int(vo[gi + 1])
        ea, eb = int(eoff[gi]), int(eoff[gi + 1])
        np.testing.assert_array_equal(res["support"][ea:eb], r1["support"])
        np.testing.assert_array_equal(res["tri"][va:vb], r1["tri"])
        np.testing.assert_array_equal(res["num"][va:vb], r1["num"])
        np.testing.assert_array_equal(res["tc"][va:vb].view(np.uint64), r1["tc"].view(np.uint64))
        assert int(res["triG"][gi]) == int(r1["triG"][0])


def test_serving_mix_equals_alone(tclib):
    from paper_2105_00110_amd import serve
    N = 60
    reqs = serve.make_requests(N, seed=11, m_lo=1e3, m_hi=3e5, workers=8)
    _say("serving", N, "requests", sum(r.pairs for r in reqs), "pairs")
    stream = torch.cuda.Stream()
    alone = [serve.run_alone(r, stream.cuda_stream) for r in reqs]
    cfg = serve.ServerConfig(budget_bytes=8 << 30, streams=4, small_pairs=1 << 15,
                             batch_pairs=1 << 18)
    srv = serve.Server(cfg)
    # all requests arrive within a few milliseconds: units queue, batch and overlap
    arrivals = serve.poisson_arrivals(N, rate=20000.0, seed=11)
    replies = srv.run(reqs, arrivals)
    _say("served", srv.stats)
    assert all(r.error is None for r in replies)
    assert srv.stats["batched_units"] > 0
    assert srv.stats["max_concurrent_units"] > 1
    assert srv.stats["peak_bytes"] <= cfg.budget_bytes
    for r in replies:
        a = alone[r.rid]
        for k in ("tri", "support", "triG", "num"):
            np.testing.assert_array_equal(r.results[k], a[k])
        np.testing.assert_array_equal(r.results["tc"].view(np.uint64), a["tc"].view(np.uint64))
    for rid in (0, 1, 2, N - 1):
        q = reqs[rid]
        _check_oracle(replies[rid].results, native.o2_paper(q.src, q.dst, q.n))


def test_serving_budget_rejects_and_bounds(tclib):
    from paper_2105_00110_amd import serve
    reqs = serve.make_requests(12, seed=21, m_lo=1e3, m_hi=1e5, workers=4)
    est = [serve.estimate_bytes([r]) for r in reqs]
    budget = sorted(est)[len(est) // 2]  # about half the requests fit alone
    cfg = serve.ServerConfig(budget_bytes=budget, streams=3, small_pairs=1, batch_pairs=1)
    srv = serve.Server(cfg)
    replies = srv.run(reqs)
    for r, e in zip(replies, est):
        if e > budget:
            assert r.error is not None
        else:
            assert r.error is None
            ref = native.o2_paper(reqs[r.rid].src, reqs[r.rid].dst, reqs[r.rid].n)
            _check_oracle(r.results, ref)
    assert srv.stats["peak_bytes"] <= budget
    assert srv.stats["rejected"] == sum(e > budget for e in est)


def test_autotune_keeps_results(tclib, tmp_path):
    from paper_2105_00110_amd import autotune
    src, dst, n = gg.rmat(14, 16, seed=14)
    ref = native.o2_paper(src, dst, n)
    g = tclib.Graph.from_edges(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(), n)
    space = {"algorithm": [1, 2], "light_max_dplus": [32, 256], "item_pairs": [128, 1024]}
    out = autotune.tune(g, space=space, reps=1, rounds=1, budget_s=60)
    tclib.tc_set_profiling(False)
    assert out["ms"] <= out["default_ms"]
    assert len(out["trials"]) >= 4
    g.compute(out["tuning"])
    _check_oracle(g.results(), ref)
    g.close()
    p = str(tmp_path / "t.json")
    autotune.store("rmat_s14", out, p)
    assert autotune.load("rmat_s14", p) == out["tuning"]


def test_serving_resident_graphs_answer_later_queries(tclib):
    # keyed requests keep their graphs resident; later top-k and vertex
    # queries on the same keys are answered from them, equal to the graph
    # run alone; a tight budget evicts and rebuilds without changing answers
    import dataclasses
    from paper_2105_00110_amd import serve
    base = serve.make_requests(6, seed=31, m_lo=2e3, m_hi=2e5, workers=6)
    stream = torch.cuda.Stream()
    alone = [serve.run_alone(r, stream.cuda_stream) for r in base]
    rng = np.random.default_rng(31)
    reqs = [dataclasses.replace(r, rid=i, key=("g", i)) for i, r in enumerate(base)]
    for j in range(24):
        i = int(rng.integers(0, len(base)))
        if j % 2:
            q = ("topk", 5)
        else:
            q = ("vertices", rng.integers(0, base[i].n, 7))
        reqs.append(dataclasses.replace(base[i], rid=len(reqs), key=("g", i), query=q))
    for budget in (8 << 30, 2 * max(serve.estimate_bytes([r]) for r in base)):
        srv = serve.Server(serve.ServerConfig(budget_bytes=budget, streams=3))
        replies = srv.run(reqs, serve.poisson_arrivals(len(reqs), 2000.0, seed=31))
        _say("resident serving, budget", budget, srv.stats)
        assert all(r.error is None for r in replies)
        assert srv.stats["resident_hits"] > 0
        for rq, rp in zip(reqs, replies):
            i = rq.key[1]
            a = alone[i]
            if rq.query[0] == "full":
                np.testing.assert_array_equal(rp.results["support"], a["support"])
                np.testing.assert_array_equal(rp.results["tc"].view(np.uint64), a["tc"].view(np.uint64))
            elif rq.query[0] == "topk":
                order = np.lexsort((np.arange(len(a["tc"])), -a["tc"]))[:5]
                np.testing.assert_array_equal(rp.results["vertices"], order)
                np.testing.assert_array_equal(rp.results["tc"].view(np.uint64), a["tc"][order].view(np.uint64))
            else:
                ids = rq.query[1]
                np.testing.assert_array_equal(rp.results["tri"].view(np.uint64), a["tri"][ids])
                np.testing.assert_array_equal(rp.results["num"].view(np.uint64), a["num"][ids])
                np.testing.assert_array_equal(rp.results["tc"].view(np.uint64), a["tc"][ids].view(np.uint64))
        srv.close()
