"""Serving loop: triangle-centrality requests on one GPU.

A request is an undirected edge list in host memory (local ids 0..n-1)
that arrives at a given time.  The server answers each with the full set of
results (tri[n], support[m] in canonical edge order, triG, num[n], tc[n])
in host memory.

How the loop works:

* Admission by device memory, in two steps.  Every request has a
  device-memory estimate from its pair and vertex counts
  (``tc_estimate_device_bytes``).  A dispatch unit starts only while the
  reservations of the units on the device stay within ``budget_bytes``.
  After the build and the orientation, a unit that goes through a handle
  asks for its exact need: the bytes the handle holds plus the bound of
  ``tc_compute_bytes``, which includes the exact size of the middle
  pivot's bit matrices (about Σ C(d+(v), 2) / 8 bytes, far above the
  estimate on dense graphs).  If the need is above the reservation and the
  difference is not free, the unit gives its memory back and its requests
  return to the head of the queue with the exact need as their estimate.
  The library's own allocator is limited to the budget as well
  (``tc_set_memory_limit``); an allocation that would pass it fails with
  TC_ERR_BUDGET and also sends the unit back to the queue (a few times at
  most).  Requests leave the queue in arrival order.  A request that cannot
  fit even alone is answered with an error and does not block the queue.
* Batching of arrivals.  Consecutive queued requests with fewer than
  ``fused_pairs`` pairs are grouped, in arrival order and up to
  ``batch_pairs`` pairs, into one fused launch (``tc_batch_fused``: one
  workgroup per graph runs the whole path, with no read-back in between);
  consecutive requests with fewer than ``small_pairs`` pairs are grouped
  into one batched handle (``tc_batch_create``), whose launches span the
  GPU.  Larger requests form units of their own with their own handle.
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
class _Reject:
    """A request larger than the whole budget: answered with an error."""

    def __init__(self, req):
        self.req = req


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
    need: int = 0         # exact device bytes, once a unit has measured them
    solo: bool = False    # sent back from a batched unit: runs alone next time
    retries: int = 0      # times sent back to the queue

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
    pairs: int = 0

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


class RequestSource:
    """Requests generated on demand, in index order, a bounded window ahead
    of the consumer: request i is made from its spec (family, m, seed) by a
    pool of host threads, and dropped by release(i) once it is answered.
    Host memory stays at about `window` requests however long the run."""

    def __init__(self, specs, window=256, workers=16):
        self.specs = list(specs)
        self.window = window
        self.ex = cf.ThreadPoolExecutor(max_workers=workers)
        self.fut = {}
        self.next_submit = 0
        self.lock = __import__("threading").Lock()

    def __len__(self):
        return len(self.specs)

    def _make(self, i):
        fam, m, seed = self.specs[i]
        src, dst, n = make_graph(fam, m, seed)
        return Request(i, src, dst, n, fam, seed)

    def _fill(self, upto):
        with self.lock:
            while self.next_submit < min(len(self.specs), upto):
                j = self.next_submit
                self.fut[j] = self.ex.submit(self._make, j)
                self.next_submit += 1

    def start(self):
        self._fill(self.window)

    def get(self, i):
        """Request i (waits for its generation)."""
        self._fill(i + self.window)
        with self.lock:
            f = self.fut[i]
        return f.result()

    def ready(self, i):
        with self.lock:
            f = self.fut.get(i)
        return f is not None and f.done()

    def release(self, i):
        with self.lock:
            self.fut.pop(i, None)

    def close(self):
        self.ex.shutdown(wait=True, cancel_futures=True)
        self.fut.clear()


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


class Requeue(Exception):
    """A unit whose exact device-memory need (``need`` bytes, 0 if
    unknown) does not fit next to the units that run: its requests go back
    to the queue."""

    def __init__(self, need=0):
        super().__init__(need)
        self.need = int(need)


def _check_need(g, tuning, admit):
    """Second admission step of a built handle: exact need = bytes held
    plus the bound of what the count allocates."""
    if admit is None:
        return
    need = g.device_bytes() + g.compute_bytes(tuning)
    if not admit(need):
        raise Requeue(need)


def run_alone(req, stream, tuning=None, keep=False, admit=None):
    """One request through its own handle: build, compute, answer.  With
    keep, returns (reply, handle) and leaves the handle open.  With admit,
    the exact need after the orientation is passed to admit(need), and
    Requeue is raised if it returns False."""
    g = tc.Graph.from_edges(req.src, req.dst, req.n, stream=stream)
    try:
        _check_need(g, tuning, admit)
        g.compute(tuning)
        out = answer(g, req.query)
    except BaseException:
        g.close()
        raise
    if keep:
        return out, g
    g.close()
    return out


# Graphs of at most this many vertices can take the fused launch
# (tc_batch_fused), which runs a whole graph per workgroup.
FUSED_MAX_N = 65535


def fused_ok(req):
    return req.n <= FUSED_MAX_N and req.key is None and req.query[0] == "full"


def run_fused(reqs, stream, fused_tuning=None):
    """Requests as one fused launch (tc_batch_fused): pairs to the device,
    one launch, results back.  Every torch operation runs on `stream`."""
    import torch
    po = np.zeros(len(reqs) + 1, np.int64)
    vo = np.zeros(len(reqs) + 1, np.int64)
    np.cumsum([r.pairs for r in reqs], out=po[1:])
    np.cumsum([r.n for r in reqs], out=vo[1:])
    src = np.concatenate([r.src for r in reqs]) if po[-1] else np.zeros(1, np.int32)
    dst = np.concatenate([r.dst for r in reqs]) if po[-1] else np.zeros(1, np.int32)
    with torch.cuda.stream(torch.cuda.ExternalStream(stream)):
        fb = tc.FusedBatch(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(), po, vo,
                           tuning=fused_tuning, stream=stream)
        fb.run()
        res = fb.results()
    out = []
    for i, r in enumerate(reqs):
        st = int(res["status"][i])
        if st < 0:
            raise tc.TCError(st, f"tc_batch_fused (request {r.rid})")
        one = fb.graph(res, i)
        out.append({"tri": one["tri"], "support": one["support"], "triG": one["triG"],
                    "num": one["num"], "tc": one["tc"]})
    return out


def run_unit(reqs, stream, tuning=None, fused_tuning=None, kind="batch", admit=None):
    """A dispatch unit: tiny requests as one fused launch (kind "fused"),
    small ones as one batched handle, a larger one through its own handle.
    admit: second admission step of handle units (see run_alone); a fused
    unit's bytes are exact from the start."""
    if kind == "fused":
        return run_fused(reqs, stream, fused_tuning)
    if len(reqs) == 1:
        return [run_alone(reqs[0], stream, tuning, admit=admit)]
    po = np.zeros(len(reqs) + 1, np.int64)
    vo = np.zeros(len(reqs) + 1, np.int64)
    np.cumsum([r.pairs for r in reqs], out=po[1:])
    np.cumsum([r.n for r in reqs], out=vo[1:])
    src = np.concatenate([r.src for r in reqs])
    dst = np.concatenate([r.dst for r in reqs])
    g = tc.Graph.batch(src, dst, po, vo, stream=stream)
    try:
        _check_need(g, tuning, admit)
        g.compute(tuning)
        res = g.results()
        eoff = g.edge_offsets()
    finally:
        g.close()
    return _split(res, reqs, vo, eoff)


def fused_bytes(reqs):
    """Device bytes of a fused unit: its workspace, the pairs and offsets,
    and the outputs."""
    P = sum(r.pairs for r in reqs)
    N = sum(r.n for r in reqs)
    G = len(reqs)
    return tc.tc_batch_fused_workspace_bytes(P, N, G) + 24 * P + 24 * N + 64 * G + (1 << 20)


def estimate_bytes(reqs, kind="batch"):
    if kind == "fused":
        return fused_bytes(reqs)
    return tc.tc_estimate_device_bytes(sum(r.pairs for r in reqs), sum(r.n for r in reqs))


# ---------------------------------------------------------------------------
# The server
# ---------------------------------------------------------------------------
@dataclass
class ServerConfig:
    budget_bytes: int = 64 << 30
    streams: int = 4
    # streams that only queries on resident graphs use: such a query takes
    # well under a millisecond and should not wait for a running build
    hit_streams: int = 1
    small_pairs: int = 1 << 17
    # requests below this many pairs go to the fused launch: one workgroup
    # per graph pays off for many tiny graphs at once, while a larger graph
    # alone is faster through a handle, whose launches span the whole GPU
    fused_pairs: int = 1 << 14
    batch_pairs: int = 1 << 22
    tuning: dict = None
    fused_tuning: dict = None
    # times a request may go back to the queue after its unit hit the
    # library's memory limit before it is answered with the error
    max_retries: int = 3


@dataclass
class _Unit:
    reqs: list
    bytes: int
    stream_idx: int = -1
    hit: object = None  # resident entry answering the request, if any
    kind: str = "batch"  # "fused" | "batch" (one request alone or a batched handle)


class Server:
    def __init__(self, cfg=None):
        import torch
        self.cfg = cfg or ServerConfig()
        self.streams = [torch.cuda.Stream()
                        for _ in range(self.cfg.streams + self.cfg.hit_streams)]
        self.stats = {"units": 0, "batched_units": 0, "batched_requests": 0, "rejected": 0,
                      "peak_bytes": 0, "max_concurrent_units": 0, "resident_hits": 0,
                      "evictions": 0, "requeued": 0, "grown": 0}
        # reservations of the running units; workers grow theirs (second
        # admission step) under the lock
        self._mu = __import__("threading").Lock()
        self._used = 0
        # cache keys whose graph a running unit is building
        self.building = {}
        # key -> {"g": handle, "bytes": device bytes, "busy": bool}, oldest first
        self.resident = collections.OrderedDict()
        self.resident_bytes = 0

    def _evict_for(self, need, free_bytes):
        """Closes least recently used idle resident graphs until need bytes
        fit; returns the new free byte count.  If closing every idle one
        would not free enough, none is closed: the unit waits for running
        units instead."""
        idle = sum(e["bytes"] for e in self.resident.values() if not e["busy"])
        if free_bytes + idle < need:
            return free_bytes
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

    def _form_unit(self, q, free_bytes, build=True):
        """Next unit to start, or None if none can start now.  Requests leave
        the queue in arrival order, with two exceptions: a request whose
        cache key is being built waits for that build (and then becomes a
        resident hit) without holding up the requests behind it, and a
        resident hit, which needs no device memory, may start ahead of a
        build that waits for memory or, with build False (no build stream
        is free), for a stream.  A build larger than the whole budget comes
        back as a _Reject of that request."""
        build_tried = not build
        for idx, r in enumerate(q):
            if r.key is not None and r.key in self.building:
                continue  # its graph is being built: answered from it later
            if r.key is not None and r.key in self.resident:
                e = self.resident[r.key]
                if e["busy"]:
                    continue
                self.resident.move_to_end(r.key)
                return _Unit([r], 0, hit=e)
            if not build_tried:
                build_tried = True
                unit = self._form_build(q, idx, free_bytes)
                if unit is not None:
                    return unit
                # the first build waits for memory: only resident hits pass it
        return None

    def _form_build(self, q, idx, free_bytes):
        """The unit that starts with the build of q[idx] (with the queued
        requests after it that batch with it), a _Reject, or None if it
        must wait for memory."""
        head = q[idx]
        est = max(estimate_bytes([head]), head.need)  # the exact need, once measured
        if est > self.cfg.budget_bytes:
            return _Reject(head)
        if est > free_bytes:
            free_bytes = self._evict_for(est, free_bytes)
            if est > free_bytes:
                return None
        if head.pairs >= self.cfg.small_pairs or not fused_ok(head) or head.solo or head.need:
            return _Unit([head], est)
        # consecutive queued requests of the head's class: tiny ones form a
        # fused launch, small ones a batched handle
        kind = "fused" if self._tiny(head) else "batch"
        reqs, pairs = [], 0
        for r in q[idx:]:
            if (r.pairs >= self.cfg.small_pairs or pairs + r.pairs > self.cfg.batch_pairs
                    or not fused_ok(r) or self._tiny(r) != (kind == "fused") or r.solo
                    or r.need):
                break
            e = estimate_bytes(reqs + [r], kind)
            if e > free_bytes:
                break
            reqs.append(r)
            pairs += r.pairs
        if not reqs:
            return _Unit([head], est)
        return _Unit(reqs, estimate_bytes(reqs, kind), kind=kind)

    def _tiny(self, r):
        return r.pairs < self.cfg.fused_pairs and fused_ok(r)

    def _admit(self, unit, need):
        """Second admission step, on a worker thread: grows the unit's
        reservation to its exact need if the difference is free."""
        with self._mu:
            extra = need - unit.bytes
            if extra <= 0:
                return True
            if self.cfg.budget_bytes - self._used - self.resident_bytes < extra:
                return False
            self._used += extra
            unit.bytes = need
            self.stats["grown"] += 1
            self.stats["peak_bytes"] = max(self.stats["peak_bytes"],
                                           self._used + self.resident_bytes)
            return True

    def run(self, requests, arrivals=None, on_reply=None):
        """Serves the requests; arrival i at arrivals[i] seconds after the start
        (all at 0 if None).  Returns replies ordered by request id.

        ``requests`` is a list or a RequestSource (requests made on demand;
        arrivals must then be non-decreasing in request id).  With
        ``on_reply``, each reply is passed to it when it is complete and its
        results are then dropped (the reply keeps its timing)."""
        source = requests if isinstance(requests, RequestSource) else None
        order = sorted(range(len(requests)),
                       key=lambda i: (arrivals[i] if arrivals is not None else 0.0, i))
        replies = [None] * len(requests)
        if source is not None:
            source.start()
            for i in range(min(len(source), source.window // 2)):
                source.get(i)  # the run starts with the first requests made
            pending = [(float(arrivals[i]) if arrivals is not None else 0.0, i) for i in order]
        else:
            pending = [(float(arrivals[i]) if arrivals is not None else 0.0, requests[i])
                       for i in order]
        self.stats["late_arrivals"] = 0
        # on_reply runs on a thread of its own, so that slow callbacks (a
        # digest of a large reply) never hold up the dispatch loop
        handoff = queue.Queue()

        def consume():
            while True:
                rep = handoff.get()
                if rep is None:
                    return
                on_reply(rep)
                rep.results = None

        consumer = None
        if on_reply is not None:
            consumer = __import__("threading").Thread(target=consume, daemon=True)
            consumer.start()

        def finish(rep):
            replies[rep.rid] = rep
            if on_reply is not None:
                handoff.put(rep)
            if source is not None:
                source.release(rep.rid)
        q = []
        # build streams, then the streams only resident hits take
        free_streams = list(range(self.cfg.streams))
        free_hit = list(range(self.cfg.streams, len(self.streams)))
        in_flight = {}
        self._used = 0
        done_q = queue.Queue()
        tc.tc_set_memory_limit(self.cfg.budget_bytes)
        t0 = time.perf_counter()

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
                    out, kept = run_alone(r0, st, self.cfg.tuning, keep=True,
                                          admit=lambda need: self._admit(unit, need))
                    res = [out]
                else:
                    res = run_unit(unit.reqs, st, self.cfg.tuning, self.cfg.fused_tuning,
                                   unit.kind, admit=lambda need: self._admit(unit, need))
                err = None
            except Requeue as e:
                res, err = None, e
            except tc.TCError as e:  # the library's memory limit: try again later
                res, err = None, (Requeue(0) if e.status == tc.TC_ERR_BUDGET else repr(e))
            except Exception as e:  # a failed unit answers its requests with the error
                res, err = None, repr(e)
            done_q.put((unit, res, err, time.perf_counter() - t0, kept))

        try:
            self._loop(pending, source, q, (free_streams, free_hit), in_flight, done_q, t0,
                       work, finish, len(requests))
        finally:
            tc.tc_set_memory_limit(0)
        self.makespan = time.perf_counter() - t0
        if consumer is not None:
            handoff.put(None)
            consumer.join()
        return replies

    def _loop(self, pending, source, q, free, in_flight, done_q, t0, work, finish, total):
        """The dispatch loop of run(); free = (free build streams, free hit
        streams)."""
        free_streams, free_hit = free
        nxt = 0
        completed = 0
        with cf.ThreadPoolExecutor(max_workers=len(self.streams)) as ex:
            while completed < total:
                now = time.perf_counter() - t0
                while nxt < len(pending) and pending[nxt][0] <= now:
                    arr, r = pending[nxt]
                    if source is not None:
                        if not source.ready(r):
                            self.stats["late_arrivals"] += 1
                        r = source.get(r)
                    r.arrival = arr
                    q.append(r)
                    nxt += 1
                while q and (free_streams or free_hit):
                    with self._mu:
                        unit = self._form_unit(
                            q, self.cfg.budget_bytes - self._used - self.resident_bytes,
                            build=bool(free_streams))
                        if isinstance(unit, _Unit):
                            self._used += unit.bytes
                            self.stats["peak_bytes"] = max(self.stats["peak_bytes"],
                                                           self._used + self.resident_bytes)
                    if unit is None:
                        break
                    if isinstance(unit, _Reject):
                        r = unit.req
                        q.remove(r)
                        finish(Reply(r.rid, None, "exceeds the device-memory budget",
                                     r.arrival, time.perf_counter() - t0, 1, r.pairs))
                        self.stats["rejected"] += 1
                        completed += 1
                        continue
                    taken = {id(r) for r in unit.reqs}
                    q[:] = [r for r in q if id(r) not in taken]
                    if unit.hit is None and unit.reqs[0].key is not None:
                        key = unit.reqs[0].key
                        self.building[key] = self.building.get(key, 0) + 1
                    unit.stream_idx = (free_hit.pop() if unit.hit is not None and free_hit
                                       else free_streams.pop())
                    if unit.hit is not None:
                        unit.hit["busy"] = True
                        self.stats["resident_hits"] += 1
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
                    if unit.hit is None and unit.reqs[0].key is not None:
                        key = unit.reqs[0].key
                        self.building[key] -= 1
                        if self.building[key] == 0:
                            del self.building[key]
                    with self._mu:
                        self._used -= unit.bytes
                    (free_streams if unit.stream_idx < self.cfg.streams
                     else free_hit).append(unit.stream_idx)
                    if unit.hit is not None:
                        unit.hit["busy"] = False
                    if kept is not None:
                        key = unit.reqs[0].key
                        if key in self.resident:  # built twice while queued: keep one
                            kept.close()
                        else:
                            b = kept.device_bytes()
                            with self._mu:
                                self.resident[key] = {"g": kept, "bytes": b, "busy": False}
                                self.resident_bytes += b
                                self.stats["peak_bytes"] = max(self.stats["peak_bytes"],
                                                               self._used + self.resident_bytes)
                    if isinstance(err, Requeue) and self._requeue(unit, err, q):
                        pass
                    else:
                        if isinstance(err, Requeue):
                            err = "exceeds the device-memory budget"
                        for i, r in enumerate(unit.reqs):
                            finish(Reply(r.rid, res[i] if res else None, err, r.arrival,
                                         t_done, len(unit.reqs), r.pairs))
                            completed += 1
                    try:
                        unit, res, err, t_done, kept = done_q.get_nowait()
                    except queue.Empty:
                        break

    def _requeue(self, unit, rq, q):
        """Puts the requests of a unit sent back by the second admission
        step at the head of the queue (their arrival order is kept: every
        queued request arrived after them).  Returns False if they are to be
        answered with the budget error instead."""
        reqs = unit.reqs
        if rq.need > self.cfg.budget_bytes and len(reqs) == 1:
            self.stats["rejected"] += 1
            return False
        for r in reqs:
            if rq.need == 0:  # the library's limit: bounded retries
                r.retries += 1
                if r.retries > self.cfg.max_retries:
                    self.stats["rejected"] += 1
                    return False
            if len(reqs) == 1:
                r.need = max(r.need, rq.need)
            else:
                r.solo = True  # each measures its own need alone
        q[0:0] = reqs
        self.stats["requeued"] += len(reqs)
        return True

    def close(self):
        """Releases every resident graph."""
        for e in self.resident.values():
            e["g"].close()
        self.resident.clear()
        self.resident_bytes = 0


def closed_loop(requests, stream, tuning=None, on_result=None):
    """One graph per launch, one at a time: returns (seconds, results list).
    With on_result(i, result) the results are handed over instead of kept
    (the list is then empty); a RequestSource is consumed in order."""
    out = []
    src = requests if isinstance(requests, RequestSource) else None
    if src is not None:
        src.start()
    busy = 0.0  # service time only: a request's generation is not counted
    for i in range(len(requests)):
        r = src.get(i) if src is not None else requests[i]
        t0 = time.perf_counter()
        res = run_alone(r, stream, tuning)
        busy += time.perf_counter() - t0
        if on_result is not None:
            on_result(i, res)
        else:
            out.append(res)
        if src is not None:
            src.release(i)
    return busy, out


def latency_by_decade(replies, warmup_frac=0.05):
    """latency_summary per decade of request size in pairs ([1e3, 1e4), ...)."""
    ok = sorted((r for r in replies if r.error is None), key=lambda r: (r.arrival, r.rid))
    ok = ok[int(len(ok) * warmup_frac):]
    out = {}
    for lo in range(3, 8):
        sel = [r for r in ok if 10 ** lo <= r.pairs < 10 ** (lo + 1)]
        if sel:
            s = latency_summary(sel, 0.0)
            out[f"1e{lo}-1e{lo + 1}"] = {k: round(v, 3) if isinstance(v, float) else v
                                         for k, v in s.items()}
    return out


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
