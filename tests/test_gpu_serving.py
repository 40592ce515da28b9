"""GPU: the batched configuration, the serving loop and the autotuner.

* 4096 Barabasi-Albert graphs with planted cliques as one batch: every
  graph bit-exact against the oracle, and the whole batch equal to one
  graph per launch on a prefix of the graphs.
* Serving: every reply of a mixed, overlapping, batched run equals the same
  request run alone (bit for bit) and the oracle, also for requests of up
  to 2e7 edges;
  graphs kept resident answer later top-k and vertex queries, also under a
  budget tight enough to evict them.
* Memory: tc_compute_bytes bounds what the count allocates; a dense request
  whose bit matrices outgrow the estimate from its pair count is refused
  under a budget below its exact need and served inside one above it.
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


def oracle_each(graphs, workers=None):
    """O2 on each (src, dst, n), one host thread per graph, graphs spread
    over the host's threads."""
    import concurrent.futures as cf
    workers = workers or native.host_threads()
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda a: native.o2_paper(a[0], a[1], a[2], nthreads=1), graphs))


def test_batched_4096_every_graph_equals_oracle(tclib, batch4096):
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
    sizes = np.diff(vo)
    assert np.all(sizes > 0)
    _say("oracle O2 on every graph")
    refs = oracle_each([(src[int(po[i]):int(po[i + 1])], dst[int(po[i]):int(po[i + 1])],
                         int(sizes[i])) for i in range(G)])
    for gi, ref in enumerate(refs):
        va, vb = int(vo[gi]), int(vo[gi + 1])
        ea, eb = int(eoff[gi]), int(eoff[gi + 1])
        one = {"support": sup[ea:eb], "tri": tri[va:vb], "triG": triG[gi:gi + 1],
               "num": num[va:vb], "tc": tcv[va:vb]}
        _check_oracle(one, ref)
        np.testing.assert_array_equal(eu[ea:eb] - va, ref.eu)
        np.testing.assert_array_equal(ev[ea:eb] - va, ref.ev)
    _say("every graph equal, triangles", int(triG.sum()))


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
    refs = oracle_each([(q.src, q.dst, q.n) for q in reqs])
    for r in replies:
        _check_oracle(r.results, refs[r.rid])


def test_serving_large_requests_equal_oracle(tclib):
    # requests up to the configuration's 2e7 edges, several above 1e6, with
    # arrivals close enough that units overlap; every reply against O2
    from paper_2105_00110_amd import serve
    N = 12
    reqs = serve.make_requests(N, seed=41, m_lo=1e5, m_hi=2e7, workers=8)
    sizes = sorted(r.pairs for r in reqs)
    _say("serving large", N, "requests, pairs", sizes)
    assert sizes[-1] > 5_000_000 and sum(p > 1_000_000 for p in sizes) >= 3
    cfg = serve.ServerConfig(budget_bytes=16 << 30, streams=4)
    srv = serve.Server(cfg)
    replies = srv.run(reqs, serve.poisson_arrivals(N, rate=200.0, seed=41))
    _say("served", srv.stats)
    assert all(r.error is None for r in replies)
    assert srv.stats["max_concurrent_units"] > 1
    assert srv.stats["peak_bytes"] <= cfg.budget_bytes
    srv.close()
    for r in replies:
        q = reqs[r.rid]
        _say("oracle request", r.rid, q.family, q.pairs)
        _check_oracle(r.results, native.o2_paper(q.src, q.dst, q.n))


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


def _clique(k):
    iu = np.triu_indices(k, 1)
    return iu[0].astype(np.int32), iu[1].astype(np.int32), k


def _check_clique(res, k):
    # K_k: every vertex on C(k-1, 2) triangles, every edge on k-2, every
    # neighbour's weight 1, so num(v) = k·C(k-1, 2) = 3·△(G) and tc = 1
    c2 = (k - 1) * (k - 2) // 2
    assert np.all(res["tri"] == c2) and np.all(res["support"] == k - 2)
    assert int(res["triG"][0]) == k * (k - 1) * (k - 2) // 6
    assert np.all(res["num"] == k * c2) and np.all(res["tc"] == 1.0)


@pytest.mark.parametrize("case", ["clique3000", "rmat16", "er_low_pivot", "batch"])
def test_compute_bytes_bounds_what_the_count_allocates(tclib, case):
    # with the cache emptied after the build, every block the count takes is
    # new: the growth of the allocator's held bytes is what it allocates
    if case == "clique3000":
        src, dst, n = _clique(3000)
        g = tclib.Graph.from_edges(src, dst, n)
    elif case == "rmat16":
        src, dst, n = gg.rmat(16, 16, seed=16)
        g = tclib.Graph.from_edges(src, dst, n)
    elif case == "er_low_pivot":
        src, dst, n = gg.er(20000, 1e-3, seed=3)
        g = tclib.Graph.from_edges(src, dst, n)
    else:
        src, dst, po, vo = gg.batched_ba(64, seed=64)
        g = tclib.Graph.batch(src, dst, po, vo)
    tclib.tc_trim_memory()
    need = g.compute_bytes()
    s0 = tclib.tc_memory_stats(reset_peaks=True)
    g.compute()
    torch.cuda.synchronize()
    s1 = tclib.tc_memory_stats()
    grown = s1["peak_held"] - s0["held"]
    _say(case, "pairs", len(src), "algorithm", g.work_stats()["algorithm"], "bound", need,
         "held growth", grown, "ratio", round(grown / need, 3))
    if case == "clique3000":
        _check_clique(g.results(), 3000)
    g.close()
    assert 0 < grown <= need


def test_dense_request_stays_inside_a_tight_budget(tclib):
    # K_3000: the bit matrices of the middle pivot (about Σ C(d+, 2) / 8
    # bytes) outgrow the estimate from the pair count; the second admission
    # step sees the exact need after the orientation
    import dataclasses

    from paper_2105_00110_amd import serve
    k = 3000
    src, dst, n = _clique(k)
    dense = serve.Request(0, src, dst, n, family="clique")
    est = serve.estimate_bytes([dense])
    g = tclib.Graph.from_edges(src, dst, n)
    need = g.device_bytes() + g.compute_bytes()
    g.close()
    _say("clique", k, "estimate", est, "exact need", need)
    assert need > est
    # a budget between the estimate and the need: the budget error, no overrun
    budget = (est + need) // 2
    tclib.tc_trim_memory()
    tclib.tc_memory_stats(reset_peaks=True)
    srv = serve.Server(serve.ServerConfig(budget_bytes=budget, streams=2))
    rep = srv.run([dense])
    _say("budget", budget, srv.stats, tclib.tc_memory_stats())
    assert rep[0].error is not None and "budget" in rep[0].error
    assert tclib.tc_memory_stats()["peak_held"] <= budget
    srv.close()
    # a budget a little above the need, with small requests arriving beside
    small = serve.make_requests(10, seed=51, m_lo=1e3, m_hi=2e5, workers=4)
    reqs = [dataclasses.replace(dense, need=0, solo=False, retries=0)] + \
        [dataclasses.replace(r, rid=i + 1) for i, r in enumerate(small)]
    budget = need + (256 << 20)
    tclib.tc_trim_memory()
    tclib.tc_memory_stats(reset_peaks=True)
    srv = serve.Server(serve.ServerConfig(budget_bytes=budget, streams=4))
    replies = srv.run(reqs)
    stats = tclib.tc_memory_stats()
    _say("budget", budget, srv.stats, stats)
    assert all(r.error is None for r in replies)
    assert stats["peak_held"] <= budget and srv.stats["peak_bytes"] <= budget
    assert srv.stats["grown"] + srv.stats["requeued"] >= 1
    srv.close()
    _check_clique(replies[0].results, k)
    for r in replies[1:]:
        q = reqs[r.rid]
        _check_oracle(r.results, native.o2_paper(q.src, q.dst, q.n))


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
    base.sort(key=lambda r: serve.estimate_bytes([r]))  # the largest graph is built last
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
    # the tight budget: the largest keyed request's estimate (keyed requests
    # keep a handle, so their estimate is the handle path's) plus half the
    # bytes the other five graphs hold once resident, so that resident
    # graphs must be evicted to build the largest, which comes last
    held = []
    for r in base:
        _, g = serve.run_alone(r, stream.cuda_stream, keep=True)
        held.append(g.device_bytes())
        g.close()
    tight = serve.estimate_bytes([reqs[len(base) - 1]]) + sum(held[:-1]) // 2
    for budget in (8 << 30, tight):
        srv = serve.Server(serve.ServerConfig(budget_bytes=budget, streams=3))
        # the six builds arrive first, 20 ms apart, then the queries
        arrivals = np.concatenate([0.02 * np.arange(len(base)),
                                   0.02 * len(base) + serve.poisson_arrivals(
                                       len(reqs) - len(base), 2000.0, seed=31)])
        replies = srv.run(reqs, arrivals)
        _say("resident serving, budget", budget, srv.stats)
        assert all(r.error is None for r in replies)
        assert srv.stats["resident_hits"] > 0
        if budget == tight:
            assert srv.stats["evictions"] > 0 and srv.stats["peak_bytes"] <= budget
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
