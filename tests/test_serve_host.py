"""Host logic of the serving loop and the autotuner (no GPU)."""
import collections
import math
import threading

import numpy as np
import pytest

from paper_2105_00110_amd import serve


def test_request_specs_mix_and_sizes():
    specs = serve.request_specs(3000, seed=5)
    fams = [f for f, _, _ in specs]
    for f in serve.FAMILIES:
        assert abs(fams.count(f) / len(fams) - 1 / 3) < 0.04
    ms = np.array([m for _, m, _ in specs], float)
    assert ms.min() >= 1e3 and ms.max() <= 2e7
    # log-uniform: log10 m is uniform on [3, log10 2e7]
    lo, hi = 3.0, math.log10(2e7)
    lg = np.log10(ms)
    assert abs(lg.mean() - (lo + hi) / 2) < 0.1
    assert [s for _, _, s in specs] == list(range(5, 5 + 3000))


def test_request_specs_deterministic():
    assert serve.request_specs(50, seed=9) == serve.request_specs(50, seed=9)


def test_poisson_arrivals():
    a = serve.poisson_arrivals(20000, rate=250.0, seed=5)
    assert a[0] == 0.0 and np.all(np.diff(a) >= 0)
    gaps = np.diff(a)
    assert abs(gaps.mean() - 1 / 250.0) < 0.05 / 250.0
    # exponential gaps: coefficient of variation 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05


@pytest.mark.parametrize("fam", serve.FAMILIES)
def test_make_graph_sizes(fam):
    src, dst, n = serve.make_graph(fam, 20000, seed=3)
    assert src.dtype == np.int32 and dst.dtype == np.int32
    assert src.min() >= 0 and dst.min() >= 0 and max(src.max(), dst.max()) < n
    assert 0.5 * 20000 <= len(src) <= 1.5 * 20000


class _R:
    def __init__(self, rid, pairs, n=10, key=None, query=("full",)):
        self.rid, self.n = rid, n
        self.src = np.zeros(pairs, np.int32)
        self.dst = np.zeros(pairs, np.int32)
        self.arrival = 0.0
        self.key, self.query = key, query
        self.need, self.solo, self.retries = 0, False, 0

    @property
    def pairs(self):
        return self.src.shape[0]


def _server(monkeypatch, **cfg):
    # a server without streams: only the unit former is exercised
    monkeypatch.setattr(serve, "estimate_bytes",
                        lambda reqs, kind="batch": 100 * sum(r.pairs for r in reqs))
    cfg.setdefault("fused_pairs", 1)  # no tiny requests unless a test asks for them
    s = serve.Server.__new__(serve.Server)
    s.cfg = serve.ServerConfig(**cfg)
    s.stats = {"evictions": 0, "grown": 0, "requeued": 0, "rejected": 0, "peak_bytes": 0}
    s.resident = collections.OrderedDict()
    s.resident_bytes = 0
    s._mu = threading.Lock()
    s._used = 0
    s.building = {}
    return s


class _G:
    def __init__(self):
        self.closed = False

    def close(self):
        self.closed = True


def test_form_unit_resident_hit_and_keyed_alone(monkeypatch):
    s = _server(monkeypatch, budget_bytes=10**9, small_pairs=100, batch_pairs=250)
    g = _G()
    s.resident["a"] = {"g": g, "bytes": 5000, "busy": False}
    s.resident_bytes = 5000
    u = s._form_unit([_R(0, 50, key="a", query=("topk", 3)), _R(1, 50)], 10**9)
    assert u.hit is s.resident["a"] and u.bytes == 0 and [r.rid for r in u.reqs] == [0]
    s.resident["a"]["busy"] = True
    assert s._form_unit([_R(0, 50, key="a")], 10**9) is None  # wait for the busy graph
    # a keyed request that is not resident is built alone, never batched
    u = s._form_unit([_R(2, 50, key="b"), _R(3, 50)], 10**9)
    assert [r.rid for r in u.reqs] == [2] and u.hit is None
    # a batch stops before a keyed request
    u = s._form_unit([_R(4, 50), _R(5, 50, key="c"), _R(6, 50)], 10**9)
    assert [r.rid for r in u.reqs] == [4]


def test_form_unit_evicts_least_recently_used(monkeypatch):
    s = _server(monkeypatch, budget_bytes=20000, small_pairs=100, batch_pairs=250)
    gs = [_G() for _ in range(3)]
    for i, g in enumerate(gs):
        s.resident[i] = {"g": g, "bytes": 6000, "busy": i == 0}
    s.resident_bytes = 18000
    # 9000 bytes needed, 2000 free: the busy oldest entry is skipped, the next two go
    u = s._form_unit([_R(0, 90)], 2000)
    assert u is not None and u.bytes == 9000
    assert [g.closed for g in gs] == [False, True, True]
    assert list(s.resident) == [0] and s.resident_bytes == 6000 and s.stats["evictions"] == 2


def test_form_unit_batches_small_in_order(monkeypatch):
    s = _server(monkeypatch, budget_bytes=10**9, small_pairs=100, batch_pairs=250)
    q = [_R(0, 50), _R(1, 90), _R(2, 99), _R(3, 40), _R(4, 500)]
    u = s._form_unit(q, 10**9)
    assert [r.rid for r in u.reqs] == [0, 1, 2]  # the next one would pass 250 pairs
    assert u.bytes == 100 * 239


def test_form_unit_tiny_and_small_do_not_mix(monkeypatch):
    # tiny requests (below fused_pairs) form a fused unit, small ones a
    # batched handle; a unit holds consecutive requests of one class
    s = _server(monkeypatch, budget_bytes=10**9, small_pairs=100, batch_pairs=250,
                fused_pairs=30)
    q = [_R(0, 10), _R(1, 29), _R(2, 60), _R(3, 5)]
    u = s._form_unit(q, 10**9)
    assert [r.rid for r in u.reqs] == [0, 1] and u.kind == "fused"
    u = s._form_unit(q[2:], 10**9)
    assert [r.rid for r in u.reqs] == [2] and u.kind == "batch"
    # a tiny request over too many vertices for the fused launch is not tiny
    big_n = _R(4, 10, n=serve.FUSED_MAX_N + 1)
    u = s._form_unit([big_n, _R(5, 10)], 10**9)
    assert [r.rid for r in u.reqs] == [4] and u.kind == "batch"


def test_form_unit_large_alone(monkeypatch):
    s = _server(monkeypatch, budget_bytes=10**9, small_pairs=100, batch_pairs=250)
    q = [_R(0, 500), _R(1, 10)]
    u = s._form_unit(q, 10**9)
    assert [r.rid for r in u.reqs] == [0]


def test_form_unit_waits_and_rejects(monkeypatch):
    s = _server(monkeypatch, budget_bytes=10000, small_pairs=100, batch_pairs=250)
    assert s._form_unit([_R(0, 90)], 8000) is None         # fits the budget, not what is free
    rj = s._form_unit([_R(0, 101)], 10000)  # larger than the whole budget
    assert isinstance(rj, serve._Reject) and rj.req.rid == 0
    u = s._form_unit([_R(0, 40), _R(1, 50)], 5000)          # the second would exceed free memory
    assert [r.rid for r in u.reqs] == [0]


def test_request_waiting_for_its_graph_does_not_block(monkeypatch):
    s = _server(monkeypatch, budget_bytes=10**9, small_pairs=100, batch_pairs=250)
    s.building = {("g", 1): 1}  # a unit is building graph ("g", 1)
    q = [_R(0, 500, key=("g", 1), query=("topk", 5)), _R(1, 500)]
    u = s._form_unit(q, 10**9)
    assert [r.rid for r in u.reqs] == [1] and u.hit is None
    s.building = {}
    g = _G()
    s.resident[("g", 1)] = {"g": g, "bytes": 10, "busy": False}
    u = s._form_unit(q, 10**9)
    assert [r.rid for r in u.reqs] == [0] and u.hit is s.resident[("g", 1)]


def test_resident_hit_passes_a_build_waiting_for_memory(monkeypatch):
    s = _server(monkeypatch, budget_bytes=10000, small_pairs=100, batch_pairs=250)
    s.resident[("g", 2)] = {"g": _G(), "bytes": 0, "busy": False}
    q = [_R(0, 90), _R(1, 90), _R(2, 5, key=("g", 2), query=("topk", 3))]
    u = s._form_unit(q, 1000)  # the first build needs 9000
    assert [r.rid for r in u.reqs] == [2] and u.hit is not None
    # a later build does not pass the first one
    assert s._form_unit(q[:2], 1000) is None


def test_without_a_free_build_stream_only_resident_hits_start(monkeypatch):
    s = _server(monkeypatch, budget_bytes=10**9, small_pairs=100, batch_pairs=250)
    s.resident[("g", 2)] = {"g": _G(), "bytes": 0, "busy": False}
    q = [_R(0, 90), _R(1, 90, key=("g", 5)), _R(2, 5, key=("g", 2), query=("topk", 3))]
    # a build stream is free: the head builds first
    assert [r.rid for r in s._form_unit(q, 10**9).reqs] == [0]
    # only the hit stream is free: the hit behind both builds starts
    u = s._form_unit(q, 10**9, build=False)
    assert [r.rid for r in u.reqs] == [2] and u.hit is not None
    assert s._form_unit(q[:2], 10**9, build=False) is None


def test_second_admission_grows_reservation_only_into_free_memory(monkeypatch):
    s = _server(monkeypatch, budget_bytes=10000, small_pairs=100, batch_pairs=250)
    u = serve._Unit([_R(0, 20)], 2000)
    s._used = 6000  # this unit's 2000 included
    s.resident_bytes = 1000
    assert s._admit(u, 1500) and u.bytes == 2000 and s._used == 6000  # below: kept
    assert s._admit(u, 5000) and u.bytes == 5000 and s._used == 9000  # 3000 free: grown
    assert not s._admit(u, 6001) and u.bytes == 5000 and s._used == 9000  # 1000 free only
    assert s.stats["grown"] == 1 and s.stats["peak_bytes"] == 10000


def test_requeue_with_exact_need(monkeypatch):
    s = _server(monkeypatch, budget_bytes=10000, small_pairs=100, batch_pairs=250)
    q = [_R(7, 10), _R(8, 10)]
    r = _R(3, 20)
    assert s._requeue(serve._Unit([r], 2000), serve.Requeue(6000), q)
    assert [x.rid for x in q] == [3, 7, 8] and r.need == 6000
    # the next unit formed reserves the exact need, alone
    assert s._form_unit(q, 5999) is None
    u = s._form_unit(q, 6000)
    assert [x.rid for x in u.reqs] == [3] and u.bytes == 6000
    # a need above the whole budget is answered with the budget error
    r2 = _R(4, 20)
    assert not s._requeue(serve._Unit([r2], 2000), serve.Requeue(10001), [])
    r2.need = 10001
    assert isinstance(s._form_unit([r2], 10000), serve._Reject)


def test_requeue_of_a_batch_runs_each_alone(monkeypatch):
    s = _server(monkeypatch, budget_bytes=10**9, small_pairs=100, batch_pairs=250)
    reqs = [_R(0, 10), _R(1, 10), _R(2, 10)]
    q = [_R(3, 10)]
    assert s._requeue(serve._Unit(reqs, 3000), serve.Requeue(9000), q)
    assert [x.rid for x in q] == [0, 1, 2, 3] and all(r.solo and r.need == 0 for r in reqs)
    assert [x.rid for x in s._form_unit(q, 10**9).reqs] == [0]


def test_requeue_after_library_limit_is_bounded(monkeypatch):
    s = _server(monkeypatch, budget_bytes=10**9, small_pairs=100, batch_pairs=250,
                max_retries=2)
    r = _R(0, 500)
    for _ in range(2):
        q = []
        assert s._requeue(serve._Unit([r], 100), serve.Requeue(0), q) and q == [r]
    assert not s._requeue(serve._Unit([r], 100), serve.Requeue(0), [])
    assert r.retries == 3


def test_latency_summary_skips_warmup():
    reps = [serve.Reply(i, {}, None, arrival=float(i), done=float(i) + (10.0 if i < 5 else 0.001))
            for i in range(100)]
    s = serve.latency_summary(reps, warmup_frac=0.05)
    assert s["measured_requests"] == 95
    assert abs(s["p99_ms"] - 1.0) < 1e-6 and abs(s["p50_ms"] - 1.0) < 1e-6


def test_digest_sensitive_to_every_array():
    base = {"tri": np.arange(4, dtype=np.uint64), "support": np.arange(3, dtype=np.uint64),
            "triG": np.array([1], np.uint64), "num": np.arange(4, dtype=np.uint64),
            "tc": np.linspace(0, 1, 4)}
    d0 = serve.digest(base)
    for k in base:
        other = {kk: vv.copy() for kk, vv in base.items()}
        other[k] = other[k].copy()
        other[k].view(np.uint8)[0] ^= 1
        assert serve.digest(other) != d0


def test_autotune_store_load(tmp_path):
    from paper_2105_00110_amd import autotune
    p = str(tmp_path / "t.json")
    assert autotune.load("w", p) is None
    autotune.store("w", {"tuning": {"item_pairs": 256}, "ms": 1.0, "default_ms": 2.0,
                         "trials": [1, 2]}, p, device="dev")
    autotune.store("v", {"tuning": {"item_pairs": 512}, "ms": 1.0, "default_ms": 2.0,
                         "trials": []}, p)
    assert autotune.load("w", p) == {"item_pairs": 256}
    assert autotune.load("v", p) == {"item_pairs": 512}
