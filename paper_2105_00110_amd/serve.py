"""Serving loop: triangle-centrality requests on one GPU.

A request is an undirected edge list in host memory (local ids 0..n-1)
that arrives at a given time.  The server answers each with the full set of
results (tri[n], support[m] in canonical edge order, triG, num[n], tc[n])
in host memory.

How the loop works:

* Admission by device memory.  Every request has a device-memory estimate
  (``tc_estimate_device_bytes``).  A dispatch unit starts only while the
  estimates of the units on the device stay within ``budget_bytes``.
  Requests leave the queue in arrival order.  A request that cannot fit
  even alone is answered with an error and does not block the queue.
* Batching of arrivals.  Queued requests with fewer than ``small_pairs``
  pairs are grouped, in arrival order and up to ``batch_pairs`` pairs, into
  one batched handle (``tc_batch_create``).  All of them are then built and
  counted by the same launches.  Larger requests form units of their own.
* Continuous batching.  ``streams`` worker threads, each with its own HIP
  stream, take units as soon as a stream and enough memory are free.
  Units that arrive while others run overlap with them on the device.
* Resident state.  The CSR, the orientation and the counts of a unit stay
  in device memory from the build to the copy of its results.  Nothing
  goes through the host in between.  A request with a cache key keeps its
  graph resident after it is answered (its device bytes count against the
  budget); later requests with the same key -- for the full results, the
  top-k vertices or the values of given vertices -- are answered from the
  resident handle without a new build or count.  Resident graphs are
  evicted least recently used when a new unit needs their memory.

The integer arithmetic is the same whether a request runs alone, in a batch
or next to other units: every result is bit-identical (tests check it).
"""
import collections
import concurrent.futures as cf
import hashlib
import math
import queue
import time
from dataclasses import dataclass

import numpy as np

from . import graphgen as gg
from . import tc

FAMILIES = ("er", "rmat", "ba")
_REJECT = object()  # head request larger than the whole budget


@dataclass
class Request:
    rid: int
    src: np.ndarray
    dst: np.ndarray
    n: int
    family: str = ""
    seed: int = 0
    arrival: float = 0.0  # seconds after the start of the run
    key: object = None    # cache key: keep the graph resident for later queries
    query: tuple = ("full",)  # ("full",) | ("topk", k) | ("vertices", ids)

    @property
    def pairs(self):
        return int(self.src.shape[0])


@dataclass
class Reply:
    rid: int
    results: dict = None
    error: str = None
    arrival: float = 0.0
    done: float = 0.0
    unit_size: int = 1

    @property
    def latency(self):
        return self.done - self.arrival


def digest(results):
    """One hash over every output array of a reply (bit patterns)."""
    h = hashlib.blake2b(digest_size=16)
    for k in ("tri", "support", "triG", "num", "tc"):
        h.update(np.ascontiguousarray(results[k]).view(np.uint8).tobytes())
    return h.hexdigest()


# ---------------------------------------------------------------------------
# Request mix
# ---------------------------------------------------------------------------
def request_specs(num, seed=5, m_lo=1e3, m_hi=2e7):
    """(family, target m, seed) per request.

    Target m is log-uniform in [m_lo, m_hi].  The family is ER, R-MAT or BA
    with probability 1/3 each.  Request i has seed ``seed + i``.
    """
    u = gg.uniform(num, seed, 0x5E)
    f = gg.uniform(num, seed, 0x5F)
    ms = np.exp(math.log(m_lo) + u * (math.log(m_hi) - math.log(m_lo)))
    fam = np.minimum((f * 3).astype(np.int64), 2)
    return [(FAMILIES[int(fam[i])], int(round(ms[i])), seed + i) for i in range(num)]


def make_graph(family, m, seed):
    """Host edge list of about m undirected edges.

    * ER: average degree 8, n = m/4, p = 8/(n-1).
    * R-MAT: (0.57, 0.19, 0.19, 0.05), scale ceil(log2(m/8)), m pairs, scrambled ids.
    * BA: attachment 4, n = m/4, no planted cliques.
    """
    if family == "er":
        n = max(16, m // 4)
        return gg.er(n, 8.0 / (n - 1), seed=seed)
    if family == "rmat":
        scale = max(4, math.ceil(math.log2(max(m, 16) / 8)))
        return gg.rmat(scale, seed=seed, num_pairs=m, nthreads=4)
    if family == "ba":
        n = max(16, m // 4)
        return gg.ba(n, 4, seed=seed, cover=0.0)
    raise ValueError(family)


def make_requests(num, seed=5, m_lo=1e3, m_hi=2e7, workers=16):
    specs = request_specs(num, seed, m_lo, m_hi)

    def one(i):
        fam, m, s = specs[i]
        src, dst, n = make_graph(fam, m, s)
        return Request(i, src, dst, n, fam, s)

    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(one, range(num)))


def poisson_arrivals(num, rate, seed=5):
    """Arrival times (s) of a Poisson process with the given rate (1/s)."""
    u = gg.uniform(num, seed, 0x5A)
    gaps = -np.log1p(-u) / rate
    return np.cumsum(gaps) - gaps[0]


# ---------------------------------------------------------------------------
# Execution of one unit
# ---------------------------------------------------------------------------
def _split(results, reqs, vtx_off, edge_off):
    out = []
    for i, r in enumerate(reqs):
        a, b = int(vtx_off[i]), int(vtx_off[i + 1])
        ea, eb = int(edge_off[i]), int(edge_off[i + 1])
        out.append({
            "tri": results["tri"][a:b],
            "support": results["support"][ea:eb],
            "triG": results["triG"][i:i + 1],
            "num": results["num"][a:b],
            "tc": results["tc"][a:b],
        })
    return out


def answer(g, query):
    """The reply to one query on a computed handle."""
    kind = query[0]
    if kind == "full":
        return g.results()
    if kind == "topk":
        verts, vals = g.top_k(int(query[1]))
        return {"vertices": verts, "tc": vals}
    if kind == "vertices":
        import torch
        ids = torch.as_tensor(np.ascontiguousarray(query[1], np.int64), device="cuda")
        r = g.results_device()
        return {k: r[k].index_select(0, ids).cpu().numpy() for k in ("tri", "num", "tc")}
    raise ValueError(f"unknown query {kind!r}")


def run_alone(req, stream, tuning=None, keep=False):
    """One request through its own handle: build, compute, answer.  With
    keep, returns (reply, handle) and leaves the handle open."""
    g = tc.Graph.from_edges(req.src, req.dst, req.n, stream=stream)
    try:
        g.compute(tuning)
        out = answer(g, req.query)
    except BaseException:
        g.close()
        raise
    if keep:
        return out, g
    g.close()
    return out


def run_unit(reqs, stream, tuning=None):
    """A dispatch unit: one request alone, or several as one batch."""
    if len(reqs) == 1:
        return [run_alone(reqs[0], stream, tuning)]
    po = np.zeros(len(reqs) + 1, np.int64)
    vo = np.zeros(len(reqs) + 1, np.int64)
    np.cumsum([r.pairs for r in reqs], out=po[1:])
    np.cumsum([r.n for r in reqs], out=vo[1:])
    src = np.concatenate([r.src for r in reqs])
    dst = np.concatenate([r.dst for r in reqs])
    g = tc.Graph.batch(src, dst, po, vo, stream=stream)
    try:
        g.compute(tuning)
        res = g.results()
        eoff = g.edge_offsets()
    finally:
        g.close()
    return _split(res, reqs, vo, eoff)


def estimate_bytes(reqs):
    return tc.tc_estimate_device_bytes(sum(r.pairs for r in reqs), sum(r.n for r in reqs))


# ---------------------------------------------------------------------------
# The server
# ---------------------------------------------------------------------------
@dataclass
class ServerConfig:
    budget_bytes: int = 64 << 30
    streams: int = 4
    small_pairs: int = 1 << 17
    batch_pairs: int = 1 << 22
    tuning: dict = None


@dataclass
class _Unit:
    reqs: list
    bytes: int
    stream_idx: int = -1
    hit: object = None  # resident entry answering the request, if any


class Server:
    def __init__(self, cfg=None):
        import torch
        self.cfg = cfg or ServerConfig()
        self.streams = [torch.cuda.Stream() for _ in range(self.cfg.streams)]
        self.stats = {"units": 0, "batched_units": 0, "batched_requests": 0, "rejected": 0,
                      "peak_bytes": 0, "max_concurrent_units": 0, "resident_hits": 0,
                      "evictions": 0}
        # key -> {"g": handle, "bytes": device bytes, "busy": bool}, oldest first
        self.resident = collections.OrderedDict()
        self.resident_bytes = 0

    def _evict_for(self, need, free_bytes):
        """Closes least recently used idle resident graphs until need bytes
        fit; returns the new free byte count."""
        for key in list(self.resident):
            if free_bytes >= need:
                break
            e = self.resident[key]
            if e["busy"]:
                continue
            e["g"].close()
            del self.resident[key]
            self.resident_bytes -= e["bytes"]
            free_bytes += e["bytes"]
            self.stats["evictions"] += 1
        return free_bytes

    def _form_unit(self, q, free_bytes):
        """Next unit from the head of the queue, or None if it must wait."""
        head = q[0]
        if head.key is not None and head.key in self.resident:
            e = self.resident[head.key]
            if e["busy"]:
                return None
            self.resident.move_to_end(head.key)
            return _Unit([head], 0, hit=e)
        est = estimate_bytes([head])
        if est > self.cfg.budget_bytes:
            return _REJECT
        if est > free_bytes:
            free_bytes = self._evict_for(est, free_bytes)
            if est > free_bytes:
                return None
        if head.pairs >= self.cfg.small_pairs or head.key is not None or head.query[0] != "full":
            return _Unit([head], est)
        reqs, pairs = [], 0
        for r in q:
            if (r.pairs >= self.cfg.small_pairs or pairs + r.pairs > self.cfg.batch_pairs
                    or r.key is not None or r.query[0] != "full"):
                break
            e = estimate_bytes(reqs + [r])
            if e > free_bytes:
                break
            reqs.append(r)
            pairs += r.pairs
        return _Unit(reqs, estimate_bytes(reqs))

    def run(self, requests, arrivals=None):
        """Serves the requests; arrival i at arrivals[i] seconds after the start
        (all at 0 if None).  Returns replies ordered by request id."""
        order = sorted(range(len(requests)),
                       key=lambda i: (arrivals[i] if arrivals is not None else 0.0, i))
        replies = [None] * len(requests)
        pending = [(float(arrivals[i]) if arrivals is not None else 0.0, requests[i]) for i in order]
        q = []
        free_streams = list(range(len(self.streams)))
        in_flight = {}
        used = 0
        done_q = queue.Queue()
        t0 = time.perf_counter()
        nxt = 0
        completed = 0

        def work(unit):
            kept = None
            try:
                st = self.streams[unit.stream_idx].cuda_stream
                r0 = unit.reqs[0]
                if unit.hit is not None:
                    g = unit.hit["g"]
                    g.stream = st
                    res = [answer(g, r0.query)]
                elif r0.key is not None:
                    out, kept = run_alone(r0, st, self.cfg.tuning, keep=True)
                    res = [out]
                else:
                    res = run_unit(unit.reqs, st, self.cfg.tuning)
                err = None
            except Exception as e:  # a failed unit answers its requests with the error
                res, err = None, repr(e)
            done_q.put((unit, res, err, time.perf_counter() - t0, kept))

        with cf.ThreadPoolExecutor(max_workers=len(self.streams)) as ex:
            while completed < len(requests):
                now = time.perf_counter() - t0
                while nxt < len(pending) and pending[nxt][0] <= now:
                    arr, r = pending[nxt]
                    r.arrival = arr
                    q.append(r)
                    nxt += 1
                while q and free_streams:
                    unit = self._form_unit(q, self.cfg.budget_bytes - used - self.resident_bytes)
                    if unit is None:
                        break
                    if unit is _REJECT:
                        r = q.pop(0)
                        replies[r.rid] = Reply(r.rid, None, "exceeds the device-memory budget",
                                               r.arrival, time.perf_counter() - t0)
                        self.stats["rejected"] += 1
                        completed += 1
                        continue
                    del q[:len(unit.reqs)]
                    unit.stream_idx = free_streams.pop()
                    if unit.hit is not None:
                        unit.hit["busy"] = True
                        self.stats["resident_hits"] += 1
                    used += unit.bytes
                    self.stats["peak_bytes"] = max(self.stats["peak_bytes"], used + self.resident_bytes)
                    self.stats["units"] += 1
                    if len(unit.reqs) > 1:
                        self.stats["batched_units"] += 1
                        self.stats["batched_requests"] += len(unit.reqs)
                    in_flight[id(unit)] = unit
                    self.stats["max_concurrent_units"] = max(self.stats["max_concurrent_units"],
                                                             len(in_flight))
                    ex.submit(work, unit)
                # wait for a completion or the next arrival
                timeout = None
                if nxt < len(pending):
                    timeout = max(0.0, pending[nxt][0] - (time.perf_counter() - t0))
                if not in_flight and timeout is None and not q:
                    break
                try:
                    unit, res, err, t_done, kept = done_q.get(timeout=timeout)
                except queue.Empty:
                    continue
                while True:
                    del in_flight[id(unit)]
                    used -= unit.bytes
                    free_streams.append(unit.stream_idx)
                    if unit.hit is not None:
                        unit.hit["busy"] = False
                    if kept is not None:
                        key = unit.reqs[0].key
                        if key in self.resident:  # built twice while queued: keep one
                            kept.close()
                        else:
                            b = kept.device_bytes()
                            self.resident[key] = {"g": kept, "bytes": b, "busy": False}
                            self.resident_bytes += b
                            self.stats["peak_bytes"] = max(self.stats["peak_bytes"],
                                                           used + self.resident_bytes)
                    for i, r in enumerate(unit.reqs):
                        replies[r.rid] = Reply(r.rid, res[i] if res else None, err, r.arrival,
                                               t_done, len(unit.reqs))
                        completed += 1
                    try:
                        unit, res, err, t_done, kept = done_q.get_nowait()
                    except queue.Empty:
                        break
        self.makespan = time.perf_counter() - t0
        return replies

    def close(self):
        """Releases every resident graph."""
        for e in self.resident.values():
            e["g"].close()
        self.resident.clear()
        self.resident_bytes = 0


def closed_loop(requests, stream, tuning=None):
    """One graph per launch, one at a time: returns (seconds, results list)."""
    out = []
    t0 = time.perf_counter()
    for r in requests:
        out.append(run_alone(r, stream, tuning))
    return time.perf_counter() - t0, out


def latency_summary(replies, warmup_frac=0.05):
    """p50/p99/mean latency in ms over the replies after the first warmup_frac
    (by arrival order), and the throughput over the whole run."""
    ok = sorted((r for r in replies if r.error is None), key=lambda r: (r.arrival, r.rid))
    skip = int(len(ok) * warmup_frac)
    lat = np.array([r.latency for r in ok[skip:]]) * 1e3
    if lat.size == 0:
        return {}
    return {
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "max_ms": float(lat.max()),
        "measured_requests": int(lat.size),
    }
