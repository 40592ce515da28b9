#!/usr/bin/env python3
"""Benchmark of the triangle-centrality hot path on one MI355X.

A step is one pass of the whole path over the R-MAT scale-24 graph
(2^28 generated pairs, (a,b,c,d) = (0.57,0.19,0.19,0.05), scrambled ids)
whose pairs are already resident in device memory: deduplication and
symmetric CSR, degree ordering, orientation, binning, intersection counting
with per-edge support, per-vertex counts and triG, Algorithm 2's
aggregation and the float64 quotient (tc_graph_from_edges + tc_compute +
tc_graph_destroy).  The metric is undirected edges (after deduplication)
per second of step time.

Printed on stdout: ONE JSON line.  Progress goes to stderr.

Beside the headline, the same JSON line carries three more workloads, each
against the plain one-graph-per-launch form on the same GPU:

* ``batched``: 4096 Barabasi-Albert graphs with planted cliques counted as
  one batch (one launch per stage for all graphs), in graphs/s;
* ``er``: Erdos-Renyi G(2000, 0.005), seeds 1..5, in microseconds per graph;
* ``served``: Poisson arrivals of mixed ER / R-MAT / BA requests (edge
  counts log-uniform in [1e3, 2e7]) through the serving loop, at 0.5x and
  0.8x of the closed-loop capacity, with p50/p99 latency and a bit-exact
  check of every served result against the same request run alone.

  python bench.py [--steps K] [--warmup W] [--scale S] [--no-cpu-baseline]
                  [--no-batched] [--no-serve] [--serve-requests N] [--autotune]
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=24)
    ap.add_argument("--tuning", type=str, default=None,
                    help="JSON file with tc_tuning knobs (default: library defaults, or "
                         "the autotuned file for this device if present)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-er", action="store_true")
    ap.add_argument("--no-ingest", action="store_true")
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="finish with a device-to-device copy of this many GiB, the known-size "
                         "kernel that scales rocprofv3's FETCH_SIZE / WRITE_SIZE readings")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the counting knobs on each workload first and store them")
    ap.add_argument("--cpu-stride", type=int, default=0,
                    help="oracle counts rows v with v %% stride == 0 (0 = automatic)")
    return ap.parse_args()


def source_digest(names):
    """Digest of the code of the given sources: comments, blank lines and
    indentation do not count, so a counter summary stays valid across
    edits that change no code."""
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2105_00110_amd", "csrc", n)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.strip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def counter_entry(kernel_key, digest):
    """The committed rocprofv3 counter summary of a kernel, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "counters_rmat_s24.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    k = d.get("kernels", {}).get(kernel_key)
    if not k or d.get("source_digest") != digest:
        return None
    return k


def cpu_baseline(src, dst, n, m, stride):
    """The oracle (O2: the paper's Procedure 2 + Algorithm 2, C, host
    threads) on a bounded sample of the same workload."""
    from oracle import native
    threads = max(1, min(16, os.cpu_count() or 1))
    phases = []
    t0 = time.perf_counter()
    native.o2_paper(src, dst, n, nthreads=threads, row_stride=stride, phases=phases)
    wall = time.perf_counter() - t0
    norm, order, count, agg = phases
    full = norm + order + count * stride + agg
    return {
        "value": m / full,
        "unit": "edges/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"O2 over all {len(src)} pairs; normalisation, ordering and aggregation "
                   f"run in full ({norm + order + agg:.1f} s), the counting loop runs on rows "
                   f"v with v % {stride} == 0 ({count:.1f} s, scaled x{stride}); "
                   f"wall {wall:.1f} s"),
        "est_full_s": full,
        "cpu_model": host_cpu_model(),
    }


def host_cpu_model():
    """The host CPU's model name, from /proc/cpuinfo (None if unreadable)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def batched_leg(args, stream, autotune):
    """4096 BA graphs: one batch vs one graph per launch (device-resident pairs)."""
    import torch
    from paper_2105_00110_amd import graphgen as gg
    from paper_2105_00110_amd import tc

    G = args.batch_graphs
    wl = f"batched_ba{G}"
    log(f"batched: generating {G} BA graphs (seed 4096)")
    src, dst, po, vo = gg.batched_ba(G, seed=4096)
    d_src = torch.from_numpy(src).cuda()
    d_dst = torch.from_numpy(dst).cuda()
    torch.cuda.synchronize()
    tuning = autotune.load(wl)
    if args.autotune:
        g = tc.Graph.batch(d_src, d_dst, po, vo, stream=stream)
        res = autotune.tune(g, log=log)
        g.close()
        autotune.store(wl, res, device=torch.cuda.get_device_name(0))
        tuning = res["tuning"]
        tc.tc_set_profiling(False)

    m = None

    def bstep():
        nonlocal m
        g = tc.Graph.batch(d_src, d_dst, po, vo, stream=stream)
        g.compute(tuning)
        if m is None:
            m = g.m
        g.close()

    bstep()
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        bstep()
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / reps
    log(f"batched: {G} graphs in {ms_batch:.2f} ms per batch")

    def single(gi):
        a, b = int(po[gi]), int(po[gi + 1])
        g = tc.Graph.from_edges(d_src[a:b], d_dst[a:b], int(vo[gi + 1] - vo[gi]), stream=stream)
        g.compute(tuning)
        g.close()

    for gi in range(min(32, G)):
        single(gi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for gi in range(G):
        single(gi)
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t0) * 1e3
    log(f"batched: one graph per launch {ms_single:.1f} ms for {G} graphs")
    return {
        "workload": wl, "graphs": G, "pairs": int(len(src)), "n": int(vo[-1]), "m": int(m),
        "ms_per_batch": round(ms_batch, 3), "graphs_per_s": G / (ms_batch / 1e3),
        "edges_per_s": m / (ms_batch / 1e3),
        "one_graph_per_launch": {"ms": round(ms_single, 3), "graphs_per_s": G / (ms_single / 1e3)},
        "speedup_vs_one_graph_per_launch": round(ms_single / ms_batch, 2),
        "tuning": tuning,
    }


def er_leg(stream, reps=20):
    """G(2000, 0.005), seeds 1..5: latency of one graph per launch, and the
    five as one batch."""
    import numpy as np
    import torch
    from paper_2105_00110_amd import graphgen as gg
    from paper_2105_00110_amd import tc

    graphs = [gg.er(2000, 0.005, seed=s) for s in range(1, 6)]
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), n) for a, b, n in graphs]
    torch.cuda.synchronize()

    def one(s, d, n):
        g = tc.Graph.from_edges(s, d, n, stream=stream)
        g.compute()
        g.close()

    for s, d, n in dev:
        one(s, d, n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for s, d, n in dev:
            one(s, d, n)
    torch.cuda.synchronize()
    us_single = (time.perf_counter() - t0) * 1e6 / (reps * len(dev))
    src = np.concatenate([g[0] for g in graphs])
    dst = np.concatenate([g[1] for g in graphs])
    po = np.zeros(len(graphs) + 1, np.int64)
    vo = np.zeros(len(graphs) + 1, np.int64)
    np.cumsum([len(g[0]) for g in graphs], out=po[1:])
    np.cumsum([g[2] for g in graphs], out=vo[1:])
    ds, dd = torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g = tc.Graph.batch(ds, dd, po, vo, stream=stream)
        g.compute()
        g.close()
    torch.cuda.synchronize()
    us_batch = (time.perf_counter() - t0) * 1e6 / (reps * len(graphs))
    log(f"er: {us_single:.1f} us per graph alone, {us_batch:.1f} us per graph in a batch of 5")
    return {"workload": "er_n2000_p0.005_seeds1-5", "us_per_graph": round(us_single, 1),
            "us_per_graph_batched5": round(us_batch, 1)}


def ingest_leg(stream):
    """A text edge list with sparse 64-bit ids (R-MAT scale 20 pairs, ids
    spread over [2^40, 2^40 + 2^20 * 1000003)): host parse, device relabel,
    then the whole path."""
    import tempfile

    import torch
    from paper_2105_00110_amd import graphgen as gg
    from paper_2105_00110_amd import tc

    s, d, _ = gg.rmat(20, 16, seed=20)
    fd, path = tempfile.mkstemp(suffix=".txt")
    os.close(fd)
    try:
        gg.write_text(path, gg.sparse_ids(s), gg.sparse_ids(d))
        size = os.path.getsize(path)
        tc.read_edge_text(path)  # page the file in once
        t0 = time.perf_counter()
        src, dst = tc.read_edge_text(path)
        t_parse = time.perf_counter() - t0
        tc.relabel(src[:1000], dst[:1000], stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s32, d32, ids, n = tc.relabel(src, dst, stream)
        t_relabel = time.perf_counter() - t0
        t0 = time.perf_counter()
        g = tc.Graph.from_edges(s32, d32, n, stream=stream)
        g.compute()
        m = g.m
        g.close()
        torch.cuda.synchronize()
        t_path = time.perf_counter() - t0
    finally:
        os.unlink(path)
    P = len(src)
    log(f"ingest: {size / 1e6:.0f} MB parsed in {t_parse * 1e3:.0f} ms, relabel {t_relabel * 1e3:.1f} ms, "
        f"path {t_path * 1e3:.1f} ms")
    return {"workload": "text_rmat_s20_sparse64_ids", "bytes": size, "pairs": P, "n": int(n),
            "m": int(m), "parse_ms": round(t_parse * 1e3, 2),
            "parse_MBps": round(size / t_parse / 1e6, 1),
            "relabel_ms_host_buffers": round(t_relabel * 1e3, 2),
            "path_ms_host_buffers": round(t_path * 1e3, 2),
            "parse_threads": os.cpu_count()}


def served_leg(args, autotune):
    """Serving loop at 0.5x and 0.8x of the closed-loop capacity."""
    import torch
    from paper_2105_00110_amd import serve

    N = args.serve_requests
    log(f"served: generating {N} requests (seed 5)")
    t0 = time.perf_counter()
    reqs = serve.make_requests(N, seed=5)
    pairs = sum(r.pairs for r in reqs)
    log(f"served: generated {pairs} pairs in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.Stream()
    for r in reqs[:8]:  # warm the path
        serve.run_alone(r, stream.cuda_stream)
    torch.cuda.synchronize()
    secs, alone = serve.closed_loop(reqs, stream.cuda_stream)
    ref = [serve.digest(a) for a in alone]
    del alone
    capacity = N / secs
    log(f"served: closed loop (one graph per launch, one at a time) {secs:.2f} s, "
        f"{capacity:.1f} graphs/s")
    cfg = serve.ServerConfig(budget_bytes=int(args.serve_budget_gb * (1 << 30)),
                             streams=args.serve_streams)
    out = {
        "workload": f"serve_mix_er_rmat_ba_m1e3-2e7_n{N}",
        "requests": N, "pairs": int(pairs),
        "budget_gb": args.serve_budget_gb, "streams": args.serve_streams,
        "small_pairs": cfg.small_pairs, "batch_pairs": cfg.batch_pairs,
        "closed_loop": {"seconds": round(secs, 3), "graphs_per_s": capacity},
        "runs": [],
    }
    for frac in (0.5, 0.8, None):
        # None: every request queued at t = 0, the server's own capacity
        rate = frac * capacity if frac else float("inf")
        arrivals = serve.poisson_arrivals(N, rate, seed=5) if frac else None
        srv = serve.Server(cfg)
        replies = srv.run(reqs, arrivals)
        ok = [r for r in replies if r.error is None]
        same = all(serve.digest(r.results) == ref[r.rid] for r in ok)
        summ = serve.latency_summary(replies)
        run = {"rate_per_s": round(rate, 2) if frac else "all at t=0",
               "load": frac if frac else "saturated", **{k: round(v, 3) if isinstance(v, float)
                                                                else v for k, v in summ.items()},
               "graphs_per_s": len(ok) / srv.makespan, "makespan_s": round(srv.makespan, 3),
               "errors": len(replies) - len(ok), "mix_equals_alone": bool(same), **srv.stats}
        log(f"served at {f'{frac}x capacity' if frac else 'saturation'}: {json.dumps(run)}")
        out["runs"].append(run)
        del replies
    out["resident"] = resident_run(reqs, cfg, capacity)
    return out


def resident_run(reqs, cfg, capacity):
    """Resident graphs: the first 200 requests are kept on the device under
    their keys; 800 further requests ask for the top-10 vertices or the
    values of 100 vertices of one of them, at 0.8x the closed-loop rate."""
    import dataclasses

    import numpy as np
    from paper_2105_00110_amd import graphgen as gg
    from paper_2105_00110_amd import serve

    K, Q = 200, 800
    base = reqs[:K]
    pick = (gg.uniform(Q, 5, 0x71) * K).astype(np.int64)
    kind = gg.uniform(Q, 5, 0x72)
    mix = [dataclasses.replace(r, rid=i, key=("g", i)) for i, r in enumerate(base)]
    for j in range(Q):
        i = int(pick[j])
        if kind[j] < 0.5:
            q = ("topk", 10)
        else:
            ids = (gg.uniform(100, 7 + j, 0x73) * base[i].n).astype(np.int64)
            q = ("vertices", ids)
        mix.append(dataclasses.replace(base[i], rid=len(mix), key=("g", i), query=q))
    rate = 0.8 * capacity
    srv = serve.Server(cfg)
    replies = srv.run(mix, serve.poisson_arrivals(len(mix), rate, seed=6))
    hits = [r for r in replies[K:] if r.error is None]
    builds = [r for r in replies[:K] if r.error is None]
    res = {"graphs": K, "queries": Q, "rate_per_s": round(rate, 2),
           "builds": {k: round(v, 3) for k, v in serve.latency_summary(builds).items()},
           "queries_on_resident": {k: round(v, 3) for k, v in serve.latency_summary(hits, 0.0).items()},
           "graphs_per_s": len(replies) / srv.makespan,
           "errors": len(replies) - len(hits) - len(builds),
           "resident_hits": srv.stats["resident_hits"], "evictions": srv.stats["evictions"],
           "resident_bytes_at_end": srv.resident_bytes}
    srv.close()
    log(f"served, resident graphs: {json.dumps(res)}")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the library "
              f"runs one graph or batch per GPU, and a sharded path is not built",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2105_00110_amd import graphgen as gg
    from paper_2105_00110_amd import tc

    torch.cuda.set_device(0)
    tc.load()
    from paper_2105_00110_amd import autotune
    wl_main = f"rmat_s{args.scale}_ef{args.edge_factor}"
    tuning = None
    if args.tuning:
        with open(args.tuning) as f:
            tuning = json.load(f).get("tuning")
    elif not args.autotune:
        tuning = autotune.load(wl_main)
    if tuning:
        log("tuning", tuning)

    log(f"generating R-MAT scale {args.scale}, edge factor {args.edge_factor}, seed {args.seed}")
    t0 = time.perf_counter()
    src, dst, n = gg.rmat(args.scale, args.edge_factor, seed=args.seed)
    log(f"generated {len(src)} pairs in {time.perf_counter() - t0:.1f} s")
    d_src = torch.from_numpy(src).cuda()
    d_dst = torch.from_numpy(dst).cuda()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream

    if args.autotune:
        g = tc.Graph.from_edges(d_src, d_dst, n, stream=stream)
        res = autotune.tune(g, log=log)
        g.close()
        autotune.store(wl_main, res, device=torch.cuda.get_device_name(0))
        tuning = res["tuning"]
        log(f"autotuned {wl_main}: {res['ms']} ms (defaults {res['default_ms']} ms)", tuning)

    tc.tc_set_profiling(True)
    stage_sum = None
    work = None
    m = None
    status = None

    def step(record):
        nonlocal stage_sum, work, m, status
        g = tc.Graph.from_edges(d_src, d_dst, n, stream=stream)
        status = g.compute(tuning)
        if record:
            ms = g.stage_ms()
            stage_sum = ms if stage_sum is None else {k: stage_sum[k] + ms[k] for k in ms}
        if work is None:
            work = g.work_stats()
            m = g.m
        g.close()

    for i in range(args.warmup):
        step(False)
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        log(f"timed step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    stages = {k: v / args.steps for k, v in stage_sum.items()}
    count_ms = sum(stages[k] for k in ("count_light", "count_heavy", "count_huge", "fold"))

    # the same step from pinned host buffers: pairs cross PCIe inside the step
    h_src = torch.from_numpy(src).pin_memory()
    h_dst = torch.from_numpy(dst).pin_memory()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = tc.Graph.from_edges(h_src.numpy(), h_dst.numpy(), n, stream=stream)
    g.compute(tuning)
    torch.cuda.synchronize()
    pcie_rate = m / (time.perf_counter() - t0)
    del h_src, h_dst
    log(f"PCIe-inclusive step: {pcie_rate:.3e} edges/s")

    # Algorithm 3's algebraic numerator on the same graph, a second device
    # path: its time, and whether it equals Algorithm 2's numerator
    alg = torch.empty(n, dtype=torch.int64, device="cuda")
    tc.tc_numerator_algebraic(g.h, alg.data_ptr(), tc.TC_MEM_DEVICE, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tc.tc_numerator_algebraic(g.h, alg.data_ptr(), tc.TC_MEM_DEVICE, stream)
    torch.cuda.synchronize()
    alg_ms = (time.perf_counter() - t0) * 1e3
    alg_equal = bool(torch.equal(alg, g.results_device()["num"]))
    g.close()
    del alg
    log(f"algebraic numerator: {alg_ms:.2f} ms, equal to Algorithm 2's: {alg_equal}")
    log("stage ms", json.dumps({k: round(v, 3) for k, v in stages.items()}))
    log("work", json.dumps(work))

    # Roofline of the dominant kernel: algorithmic bytes per launch = the
    # streamed candidates (4 B each, 2 B for those read as 16-bit entries:
    # pivots among the top 2^16 ranks) + 8 B per scanned pair (its in-pair
    # word) + 8 B per pivot row (row offsets).
    bins = {"count_light": "light", "count_heavy": "heavy", "count_huge": "huge"}
    dom = max(bins, key=lambda k: stages[k])
    b = bins[dom]
    c16 = work.get(f"cand_{b}_16", 0)
    algo_bytes = (4 * (work[f"cand_{b}"] - c16) + 2 * c16 + 8 * work[f"edges_{b}"]
                  + 8 * work[f"rows_{b}"])
    dur_s = stages[dom] / 1e3
    achieved = algo_bytes / dur_s / 1e9 if dur_s > 0 else 0.0
    digest = source_digest(["tc_count.hip", "tc_count_mid.hip", "tc_table.h", "tc_internal.h"])
    counters = counter_entry(dom, digest) or {}
    kernel_names = {"count_light": "k_mid_wave", "count_heavy": "k_mid_block",
                    "count_huge": "k_mid_block<true>"}
    if work.get("algorithm") == 1:
        kernel_names = {"count_light": "k_count_light", "count_heavy": "k_count_heavy",
                        "count_huge": "k_count_heavy<true>"}
    roofline = {
        "bound": "hbm",
        "kernel": kernel_names[dom],
        "stage": dom,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": counters.get("hbm_bytes_per_dispatch"),
        "algorithmic_bytes": int(algo_bytes),
        "avg_ms": round(stages[dom], 3),
        # fraction of cycles the SIMDs issued vector ALU work, from the same
        # counter summary (null when it is stale)
        "valu_busy": counters.get("valu_busy"),
    }

    result = {
        "metric": "TC edges/s, R-MAT scale 24 (whole hot path, device-resident pairs)",
        "value": m / (ms_per_step / 1e3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 integer counts, f64 quotient",
        "data": "synthetic",
        "config": {
            "workload": f"rmat_s{args.scale}_ef{args.edge_factor}",
            "scale": args.scale, "edge_factor": args.edge_factor, "seed": args.seed,
            "abcd": [0.57, 0.19, 0.19, 0.05], "pairs": int(len(src)), "n": int(n), "m": int(m),
            "triangles": work["triangles"], "tuning": tuning, "status": status,
        },
        "stages_ms": {k: round(v, 3) for k, v in stages.items()},
        "count_plus_aggregate_edges_per_s": m / (sum(stages[k] for k in
                                                   ["bin", "count_light", "count_heavy",
                                                    "count_huge", "tri", "aggregate"]) / 1e3),
        "work": work,
        "roofline": roofline,
        # the count priced in the low-pivot form, 4 B per candidate of
        # W_hash = sum over v->u of |N_H(u)|, over the whole count stage
        "hash_form_algorithmic_count": {
            "bytes": 4 * work["w_hash"], "ms": round(count_ms, 3),
            "GBps": round(4 * work["w_hash"] / (count_ms / 1e3) / 1e9, 1),
            "frac_of_peak": round(4 * work["w_hash"] / (count_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        },
        "pcie_inclusive_edges_per_s": pcie_rate,
        "algebraic_numerator": {"ms": round(alg_ms, 3), "equals_algorithm2": alg_equal,
                                "aggregate_ms": round(stages["aggregate"], 3)},
    }

    del d_src, d_dst
    torch.cuda.empty_cache()
    tc.tc_set_profiling(False)
    if not args.no_batched:
        result["batched"] = batched_leg(args, stream, autotune)
    if not args.no_er:
        result["er"] = er_leg(stream)
    if not args.no_ingest:
        result["ingest"] = ingest_leg(stream)
    if not args.no_serve:
        result["served"] = served_leg(args, autotune)

    if not args.no_cpu_baseline:
        stride = args.cpu_stride or max(1, 1 << max(0, args.scale - 20))
        log(f"CPU baseline: oracle O2 with row stride {stride}")
        cb = cpu_baseline(src, dst, n, m, stride)
        result["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample",
                                                      "cpu_model")}
        log(f"CPU baseline done: {cb['value']:.3e} edges/s, est. full {cb['est_full_s']:.1f} s")
    if args.copy_calibration > 0:
        nbytes = int(args.copy_calibration * (1 << 30))
        a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(7)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = nbytes
        log(f"copy calibration: 3 copies of {nbytes} bytes")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
