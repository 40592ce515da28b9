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

* ``batched``: 4096 Barabasi-Albert graphs with planted cliques counted by
  one persistent fused launch (and by its replay from a captured graph), in
  graphs/s;
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
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-poisson", type=int, default=3000,
                    help="requests of the Poisson runs (the first ones of the mix)")
    ap.add_argument("--serve-saturated", type=int, default=1000,
                    help="requests queued at t = 0 in the saturated run")
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="finish with a device-to-device copy of this many GiB, the known-size "
                         "kernel that scales rocprofv3's FETCH_SIZE / WRITE_SIZE readings")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the counting knobs on each workload first and store them")
    ap.add_argument("--cpu-stride", type=int, default=0,
                    help="oracle counts rows v with v %% stride == 0 (0 = automatic)")
    ap.add_argument("--summarize-counters", type=str, default=None, metavar="DIR",
                    help="no GPU work: turn the rocprofv3 CSVs under DIR (pmc_1/, pmc_2/, "
                         "ktrace/) into profiles/counters_rmat_s24.{json,md}")
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


# Counter passes of the summary (one rocprofv3 run each; each within the
# per-block limits of one pass).  HBM bytes come from the L2's requests to
# memory counted by request size: reads of 32 and 64 bytes and whole
# 128-byte lines (the rest), writes of 64 bytes and of 32 bytes (the rest).  A device-to-device copy of known
# size checks the rule: its bytes must come out exact.
PMC_PASSES = [
    ["TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum",
     "TCC_EA0_RDREQ_128B_sum", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU", "SQ_WAVES",
     "GRBM_GUI_ACTIVE"],
    ["TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum", "TCC_HIT_sum", "TCC_MISS_sum", "SQ_INSTS_LDS",
     "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS", "SQ_INSTS_VMEM_RD"],
    # the requests the L2 sends on to DRAM, beside all of its requests (a
    # request the MALL serves would show as the difference)
    ["TCC_EA0_RDREQ_DRAM_sum", "TCC_EA0_WRREQ_DRAM_sum", "TCC_EA0_RDREQ_sum", "TCC_EA0_WRREQ_sum"],
]
# kernels of the summary: (short name, which of its launch shapes in launch
# order, or None for all) -> stage
COUNTER_KERNELS = [
    ("k_mid_block16", None, "count_heavy"), ("k_mid_block<2>", None, "count_light_bitmap"),
    ("k_mid_wave", None, "count_light"), ("k_mid_groups<16>", None, "count_light_groups"),
    ("k_fold_big<int>", None, "fold_big"), ("k_fold<16>", None, "fold_small"),
    ("k_place_by_smaller", None, "orient_place_smaller"),
    ("k_place_by_larger", None, "orient_place_larger"),
    ("k_orient_small", None, "orient_sort_small"), ("k_orient_mid", None, "orient_sort_mid"),
    ("k_unique_emit", None, "csr_unique_emit"), ("k_rank_rows<1>", None, "tri_rows"),
    ("k_rank_chunks<1>", None, "tri_chunks"), ("k_rank_rows<2>", None, "aggregate_rows"),
    ("k_rank_chunks<2>", None, "aggregate_chunks"),
    ("__amd_rocclr_copyBuffer", None, "copy_calibration"),
]
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COUNTER_REGEX = "k_mid_block|k_mid_wave|k_mid_groups|k_fold|copyBuffer|k_place_by|k_orient_small|" \
                "k_orient_mid|k_unique_emit|k_rank_rows|k_rank_chunks"
COUNTER_ARGS = "--steps 1 --warmup 0 --no-batched --no-serve --no-er --no-ingest " \
               "--no-cpu-baseline --copy-calibration 1"
COUNT_SOURCES = ["tc_count.hip", "tc_count_mid.hip", "tc_table.h", "tc_internal.h"]


def _short_kernel(name):
    name = re.sub(r"\(.*", "", name.replace("(anonymous namespace)::", ""))
    name = name.replace("void ", "").replace("int32_t", "int").strip()
    return re.sub(r"\s+", "", name)


def _csv_rows(d, suffix):
    import csv
    import glob
    out = []
    for f in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(f) as fh:
            out.extend(csv.DictReader(fh))
    return out


def summarize_counters(d, out_dir=None):
    """profiles/counters_rmat_s24.{json,md} (or in out_dir) from the
    rocprofv3 runs under d."""
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    import collections
    per = collections.defaultdict(lambda: collections.defaultdict(dict))  # key -> dispatch -> c
    first = {}
    for i in range(len(PMC_PASSES)):
        for r in _csv_rows(os.path.join(d, f"pmc_{i + 1}"), "counter_collection.csv"):
            short = _short_kernel(r["Kernel_Name"])
            key = (short, int(r["Grid_Size"]))
            disp = int(r.get("Dispatch_Id") or 0)
            first[key] = min(first.get(key, disp), disp) if i == 0 else first.get(key, disp)
            per[key][(i, disp)][r["Counter_Name"]] = float(r["Counter_Value"])
    stats = {}
    for r in _csv_rows(os.path.join(d, "ktrace"), "kernel_stats.csv"):
        stats[_short_kernel(r["Name"])] = float(r["AverageNs"]) / 1e6
    # mean duration per launch shape, from the kernel trace of the same run
    dur = collections.defaultdict(list)
    copy_dur = []
    for r in _csv_rows(os.path.join(d, "ktrace"), "kernel_trace.csv"):
        grid = 1
        for ax in "XYZ":
            grid *= int(r.get(f"Grid_Size_{ax}") or 1)
        short = _short_kernel(r["Kernel_Name"])
        ms = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        dur[(short, grid)].append(ms)
        if short == COPY_KERNEL:
            copy_dur.append((int(r.get("Dispatch_Id") or 0), ms))
    shapes = collections.defaultdict(list)
    for (short, grid) in sorted(per, key=lambda k: first.get(k, 0)):
        shapes[short].append(grid)

    def mean(key, counter):
        vals = [c[counter] for c in per[key].values() if counter in c]
        return sum(vals) / len(vals) if vals else 0.0

    # the calibration copy: the last three copy dispatches (the benchmark's
    # final step), told apart from the library's smaller copies of the same
    # launch shape by dispatch order
    copies = sorted(((disp, key) for key in per if key[0] == COPY_KERNEL
                     for (i, disp) in per[key] if i == 0))[-3:]
    copy_disp = {d for d, _ in copies}

    kernels = {}
    for short, idx, stage in COUNTER_KERNELS:
        grids = shapes.get(short, [])
        if not grids or (idx is not None and idx >= len(grids)):
            continue
        sel = grids if idx is None else [grids[idx]]
        keys = [(short, g) for g in sel]

        def tot(counter):
            if short == COPY_KERNEL:
                vals = [c[counter] for k in keys for (i, d), c in per[k].items()
                        if d in copy_disp and counter in c]
                return sum(vals) / len(vals) if vals else 0.0
            return sum(mean(k, counter) for k in keys) / len(keys)
        rd, r32 = tot("TCC_EA0_RDREQ_sum"), tot("TCC_EA0_RDREQ_32B_sum")
        r64, r128 = tot("TCC_EA0_RDREQ_64B_sum"), tot("TCC_EA0_RDREQ_128B_sum")
        wr, w64 = tot("TCC_EA0_WRREQ_sum"), tot("TCC_EA0_WRREQ_64B_sum")
        rbytes = 32 * r32 + 64 * r64 + 128 * (rd - r32 - r64)
        wbytes = 64 * w64 + 32 * (wr - w64)
        gui = tot("GRBM_GUI_ACTIVE")
        hit, miss = tot("TCC_HIT_sum"), tot("TCC_MISS_sum")
        lds_active = tot("SQ_ACTIVE_INST_LDS")
        ds = [t for k in keys for t in dur.get(k, [])] if short != COPY_KERNEL else \
            [t for _, t in sorted(copy_dur)[-3:]]
        e = {
            "kernel": f"{short}@{sel[0]}" if idx is not None else short,
            "avg_ms": round(sum(ds) / len(ds), 4) if ds else None,
            "trace_dispatches": len(ds),
            "rdreq": int(rd), "rdreq_32b": int(r32), "rdreq_64b": int(r64),
            "rdreq_128b": int(r128), "rdreq_unsized": int(rd - r32 - r64 - r128),
            "wrreq": int(wr), "wrreq_64b": int(w64),
            "hbm_read_bytes": int(rbytes), "hbm_write_bytes": int(wbytes),
            "hbm_bytes_per_dispatch": int(rbytes + wbytes),
            "valu_insts": int(tot("SQ_INSTS_VALU")),
            "valu_busy": round(tot("SQ_ACTIVE_INST_VALU") * 4 / (4 * 256 * gui / 8), 3)
            if gui else None,
            "lds_insts": int(tot("SQ_INSTS_LDS")),
            "lds_bank_conflict_per_active_lds_cycle":
                round(tot("SQ_LDS_BANK_CONFLICT") / lds_active, 3) if lds_active else None,
            "vmem_rd_insts": int(tot("SQ_INSTS_VMEM_RD")),
            "tcc_hit_rate": round(hit / (hit + miss), 3) if hit + miss else None,
            "rdreq_dram_fraction": round(tot("TCC_EA0_RDREQ_DRAM_sum") / rd, 4) if rd else None,
            "wrreq_dram_fraction": round(tot("TCC_EA0_WRREQ_DRAM_sum") / wr, 4) if wr else None,
            "gpu_cycles_per_xcd": int(gui / 8),
            "dispatches": sum(1 for k in keys for (i, _) in per[k] if i == 0),
        }
        kernels[stage] = e
    for stage, e in kernels.items():
        short = e["kernel"].split("@")[0]
        e["stats_avg_ms_all_shapes"] = round(stats[short], 4) if short in stats else None
    for e in kernels.values():
        if e["avg_ms"]:
            e["hbm_GBps"] = round(e["hbm_bytes_per_dispatch"] / (e["avg_ms"] / 1e3) / 1e9, 1)
    cal = kernels.get("copy_calibration")
    check = None
    if cal:
        nbytes = 1 << 30
        check = {"bytes_read": nbytes, "bytes_written": nbytes,
                 "counted_read": cal["hbm_read_bytes"], "counted_written": cal["hbm_write_bytes"],
                 "read_ratio": round(cal["hbm_read_bytes"] / nbytes, 5),
                 "write_ratio": round(cal["hbm_write_bytes"] / nbytes, 5)}
    cmds = counter_commands()
    out = {"source_digest": source_digest(COUNT_SOURCES),
           "workload": "rmat_s24_ef16 seed 24, tuning from "
                       "paper_2105_00110_amd/tuning/mi355x.json",
           "rule": "read bytes = 32 x TCC_EA0_RDREQ_32B + 64 x TCC_EA0_RDREQ_64B + 128 x "
                   "(the other TCC_EA0_RDREQ, whole-line fills, which TCC_EA0_RDREQ_128B "
                   "counts when it does); write bytes = 64 x TCC_EA0_WRREQ_64B + 32 x "
                   "(TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B); no scale factor",
           "copy_check": check, "commands": cmds, "kernels": kernels}
    with open(os.path.join(out_dir, "counters_rmat_s24.json"), "w") as f:
        json.dump(out, f, indent=1)
    lines = ["# Hardware counters, R-MAT scale 24 (edge factor 16, seed 24)", "",
             "Made by these commands (one MI355X, from the repository root; the last line "
             "runs on any host):", "", "```"] + cmds + ["```", "",
             "## Rule, checked on a copy of known size", "",
             f"- {out['rule']}.",
             "- On the copy, read requests by size: "
             f"{cal['rdreq_32b'] if cal else 'n/a'} of 32 B, "
             f"{cal['rdreq_64b'] if cal else 'n/a'} of 64 B, "
             f"{cal['rdreq_128b'] if cal else 'n/a'} of 128 B, "
             f"{cal['rdreq_unsized'] if cal else 'n/a'} not in any of the three. FETCH_SIZE "
             "takes 128-byte fills from TCC_BUBBLE and prices every other request at 64 B.",
             f"- 1 GiB device-to-device copy: counted read / true = "
             f"{check['read_ratio'] if check else 'n/a'}, counted written / true = "
             f"{check['write_ratio'] if check else 'n/a'}.",
             "- The DRAM share is TCC_EA0_RDREQ_DRAM / TCC_EA0_RDREQ (and the same for writes). "
             "A share of 1 means the counter reports every L2 miss as a DRAM request, so on this "
             "device it cannot tell requests the 256 MB MALL serves from those HBM serves: the "
             "bytes above are L2-miss bytes, which can run above the copy rate.", "",
             "## Per kernel (mean per dispatch)", "",
             "| stage | kernel | ms | read GB | reads 128 B / 64 B / 32 B (M) | write GB | "
             "HBM GB/s | DRAM share of read / write requests | VALU busy | L2 hit | "
             "LDS conflicts / active LDS cycle |",
             "|---|---|---:|---:|---|---:|---:|---|---:|---:|---:|"]
    for stage, e in kernels.items():
        mix = (f"{(e['rdreq'] - e['rdreq_64b'] - e['rdreq_32b']) / 1e6:.1f} / "
               f"{e['rdreq_64b'] / 1e6:.1f} / {e['rdreq_32b'] / 1e6:.1f}")
        lines.append(f"| {stage} | `{e['kernel']}` | {e['avg_ms'] or ''} | "
                     f"{e['hbm_read_bytes'] / 1e9:.2f} | {mix} | {e['hbm_write_bytes'] / 1e9:.2f} | "
                     f"{e.get('hbm_GBps', '')} | {e['rdreq_dram_fraction']} / "
                     f"{e['wrreq_dram_fraction']} | {e['valu_busy']} | {e['tcc_hit_rate']} | "
                     f"{e['lds_bank_conflict_per_active_lds_cycle']} |")
    lines += ["", f"Source digest of the counting sources: `{out['source_digest']}`. "
              "`bench.py` reports `traffic` from this file only while it matches.", ""]
    with open(os.path.join(out_dir, "counters_rmat_s24.md"), "w") as f:
        f.write("\n".join(lines))
    print(json.dumps({k: {kk: v[kk] for kk in ("avg_ms", "hbm_bytes_per_dispatch")}
                      for k, v in kernels.items()}, indent=1))


def counter_commands():
    cmds = ["cd /tmp && export TMPDIR=/tmp"]
    for i, p in enumerate(PMC_PASSES):
        cmds.append(f"timeout -s KILL 240 rocprofv3 --pmc {' '.join(p)} --kernel-include-regex "
                    f"'{COUNTER_REGEX}' -d /root/repo/gpurun_out/pmc_s24/pmc_{i + 1} -o run "
                    f"--output-format csv -- python3 /root/repo/bench.py {COUNTER_ARGS}")
    cmds.append("timeout -s KILL 300 rocprofv3 --kernel-trace --stats -d "
                "/root/repo/gpurun_out/pmc_s24/ktrace -o run --output-format csv -- python3 "
                "/root/repo/bench.py --steps 3 --warmup 1 --no-batched --no-serve --no-er "
                "--no-ingest --no-cpu-baseline --copy-calibration 1")
    cmds.append("cd /root/repo && python3 bench.py --summarize-counters gpurun_out/pmc_s24")
    return cmds


def cpu_baseline(src, dst, n, m, stride):
    """The oracle (O2: the paper's Procedure 2 + Algorithm 2, C, host
    threads) on a bounded sample of the same workload, on the host threads a
    GPU machine grants one process (at most 16), and once more on one thread."""
    from oracle import native
    threads = native.host_threads()
    phases = []
    t0 = time.perf_counter()
    native.o2_paper(src, dst, n, nthreads=threads, row_stride=stride, phases=phases)
    wall = time.perf_counter() - t0
    norm, order, count, agg = phases
    full = norm + order + count * stride + agg
    # one thread: the same normalisation, ordering and aggregation (they are
    # single-threaded in the oracle), the counting loop on a 16x sparser
    # sample of rows
    stride1 = stride * 16
    ph1 = []
    native.o2_paper(src, dst, n, nthreads=1, row_stride=stride1, phases=ph1)
    full1 = ph1[0] + ph1[1] + ph1[2] * stride1 + ph1[3]
    return {
        "value": m / full,
        "unit": "edges/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"O2 over all {len(src)} pairs; normalisation, ordering and aggregation "
                   f"run in full ({norm + order + agg:.1f} s), the counting loop runs on rows "
                   f"v with v % {stride} == 0 ({count:.1f} s on {threads} threads, scaled "
                   f"x{stride}); wall {wall:.1f} s"),
        "est_full_s": full,
        "single_thread": {"edges_per_s": m / full1, "est_full_s": round(full1, 1),
                          "sample": f"counting loop on rows v % {stride1} == 0, scaled "
                                    f"x{stride1} ({ph1[2]:.1f} s)"},
        "host_cpus": os.cpu_count(),
        "cpu_model": host_cpu_model(),
    }


def host_cpu_model():
    """The host CPU's model name, family, model and stepping numbers and
    socket/core layout from /proc/cpuinfo (None if unreadable)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("model name", "cpu family", "model", "stepping", "cpu cores",
                         "siblings", "cpu MHz") and k not in info:
                    info[k] = v
    except OSError:
        return None
    if "model name" not in info:
        return None
    return (f"{info['model name']} (family {info.get('cpu family')}, model {info.get('model')}, "
            f"stepping {info.get('stepping')}; {info.get('cpu cores')} cores / "
            f"{info.get('siblings')} threads per socket; {info.get('cpu MHz')} MHz)")


def _event_ms(fn, reps):
    """Median device time (ms) of fn() over reps, by HIP events on torch's
    current stream (the stream the fused launch is queued on)."""
    import torch
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def _graph_replay_ms(fb, reps):
    """The fused launch captured once in a graph, then replayed: median
    device time (ms) of one replay, and the wall time (us) of a replay plus
    its synchronisation."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    saved = fb.stream
    fb.stream = side.cuda_stream
    with torch.cuda.stream(side):
        fb.run()
    torch.cuda.synchronize()
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg, stream=side):
        fb.run()
    torch.cuda.synchronize()
    fb.stream = saved
    ms = _event_ms(cg.replay, reps)
    t0 = time.perf_counter()
    for _ in range(reps):
        cg.replay()
        torch.cuda.synchronize()
    wall_us = (time.perf_counter() - t0) * 1e6 / reps
    return ms, wall_us


def batched_leg(args, stream, autotune):
    """4096 BA graphs: the fused launch (one persistent kernel for the whole
    batch, also replayed from a captured graph) against one graph per launch,
    and against the batch as one handle (every stage one launch over the
    disjoint union)."""
    import numpy as np
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
    ft = autotune.load(wl + "_fused")
    if args.autotune:
        res = autotune.tune_fused(d_src, d_dst, po, vo, log=log)
        autotune.store(wl + "_fused", res, device=torch.cuda.get_device_name(0))
        ft = res["tuning"]
    ft = ft or {"order": "largest_first"}
    order = ft.get("order", "largest_first")
    fknobs = {k: v for k, v in ft.items() if k in ("block", "wg_per_cu")} or None
    fb = tc.FusedBatch(d_src, d_dst, po, vo, order=order, tuning=fknobs, stream=stream)
    fb.run()
    torch.cuda.synchronize()
    st = fb.status.cpu().numpy()
    m = int(fb.num_edges.cpu().numpy().sum())
    ms_fused = _event_ms(fb.run, 5)
    ms_graph, _ = _graph_replay_ms(fb, 5)
    log(f"batched: fused launch {ms_fused:.2f} ms per batch, graph replay {ms_graph:.2f} ms, "
        f"statuses {np.unique(st).tolist()}")
    del fb

    tuning = autotune.load(wl)

    def union():
        g = tc.Graph.batch(d_src, d_dst, po, vo, stream=stream)
        g.compute(tuning)
        g.close()

    union()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        union()
    torch.cuda.synchronize()
    ms_union = (time.perf_counter() - t0) * 1e3 / 3
    log(f"batched: one handle over the disjoint union {ms_union:.2f} ms per batch")

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
        "workload": wl, "graphs": G, "pairs": int(len(src)), "n": int(vo[-1]), "m": m,
        "fused_launch": {"ms_per_batch": round(ms_fused, 3), "graphs_per_s": G / (ms_fused / 1e3),
                         "edges_per_s": m / (ms_fused / 1e3), "tuning": ft,
                         "graph_replay_ms": round(ms_graph, 3)},
        "ms_per_batch": round(ms_fused, 3), "graphs_per_s": G / (ms_fused / 1e3),
        "one_handle_union": {"ms": round(ms_union, 3), "graphs_per_s": G / (ms_union / 1e3)},
        "one_graph_per_launch": {"ms": round(ms_single, 3), "graphs_per_s": G / (ms_single / 1e3)},
        "speedup_vs_one_graph_per_launch": round(ms_single / ms_fused, 2),
        "tuning": tuning,
    }


def er_leg(stream, reps=20):
    """G(2000, 0.005), seeds 1..5: latency of one graph per launch (a handle;
    the fused launch; the fused launch replayed from a captured graph), and
    the five as one fused launch."""
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
    fbs = [tc.FusedBatch(s, d, [0, len(s)], [0, n], stream=stream) for s, d, n in dev]
    for fb in fbs:
        fb.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for fb in fbs:
            fb.run()
            torch.cuda.synchronize()
    us_fused = (time.perf_counter() - t0) * 1e6 / (reps * len(fbs))
    us_fused_dev = np.mean([_event_ms(fb.run, reps) for fb in fbs]) * 1e3
    replay = [_graph_replay_ms(fb, reps) for fb in fbs]
    us_replay_dev = np.mean([r[0] for r in replay]) * 1e3
    us_replay_wall = np.mean([r[1] for r in replay])
    src = np.concatenate([g[0] for g in graphs])
    dst = np.concatenate([g[1] for g in graphs])
    po = np.zeros(len(graphs) + 1, np.int64)
    vo = np.zeros(len(graphs) + 1, np.int64)
    np.cumsum([len(g[0]) for g in graphs], out=po[1:])
    np.cumsum([g[2] for g in graphs], out=vo[1:])
    fb5 = tc.FusedBatch(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(), po, vo,
                        stream=stream)
    us_batch = _event_ms(fb5.run, reps) * 1e3 / len(graphs)
    log(f"er: one handle {us_single:.1f} us per graph; fused launch {us_fused:.1f} us "
        f"(device {us_fused_dev:.1f}); graph replay {us_replay_wall:.1f} us (device "
        f"{us_replay_dev:.1f}); five in one fused launch {us_batch:.1f} us per graph")
    return {"workload": "er_n2000_p0.005_seeds1-5",
            "us_per_graph": round(us_fused, 1),
            "us_per_graph_one_handle": round(us_single, 1),
            "us_per_graph_fused_device": round(us_fused_dev, 1),
            "us_per_graph_graph_replay": round(us_replay_wall, 1),
            "us_per_graph_graph_replay_device": round(us_replay_dev, 1),
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
    """Serving loop.  The closed loop (one graph per launch, one at a time)
    runs all N requests, made from their seeds a bounded window ahead, and
    keeps a digest of each result; its service time gives the capacity.
    Then Poisson arrivals at 0.8x and 0.5x of that capacity, and every
    request at t = 0, over the first --serve-poisson requests (made before
    the runs): each reply is compared, by digest, with the same request run
    alone, and then dropped."""
    import torch
    from paper_2105_00110_amd import serve

    N = args.serve_requests
    specs = serve.request_specs(N, seed=5)
    pairs = sum(m for _, m, _ in specs)
    log(f"served: {N} requests (seed 5), {pairs} pairs, made on demand")
    stream = torch.cuda.Stream()
    for r in serve.make_requests(8, seed=5):  # warm the path
        serve.run_alone(r, stream.cuda_stream)
    torch.cuda.synchronize()
    ref = [None] * N

    def keep_digest(i, res):
        ref[i] = serve.digest(res)
        if (i + 1) % 1000 == 0:
            log(f"served: closed loop {i + 1}/{N}")

    src = serve.RequestSource(specs)
    secs, _ = serve.closed_loop(src, stream.cuda_stream, on_result=keep_digest)
    src.close()
    capacity = N / secs
    log(f"served: closed loop (one graph per launch, one at a time) {secs:.2f} s of service, "
        f"{capacity:.1f} graphs/s")
    cfg = serve.ServerConfig(budget_bytes=int(args.serve_budget_gb * (1 << 30)),
                             streams=args.serve_streams)
    out = {
        "workload": f"serve_mix_er_rmat_ba_m1e3-2e7_n{N}",
        "requests": N, "pairs": int(pairs),
        "budget_gb": args.serve_budget_gb, "streams": args.serve_streams, "hit_streams": cfg.hit_streams,
        "small_pairs": cfg.small_pairs, "batch_pairs": cfg.batch_pairs,
        "closed_loop": {"seconds": round(secs, 3), "graphs_per_s": capacity},
        "runs": [],
    }
    # the Poisson and saturated runs take the first --serve-poisson requests,
    # made before the run: making requests while serving takes the host CPUs
    # the server needs, and all 10,000 would hold 164 GB of pairs
    Np = min(N, args.serve_poisson)
    log(f"served: making the first {Np} requests for the Poisson runs")
    pre = serve.make_requests(Np, seed=5)
    for frac, count in ((0.8, Np), (0.5, Np), (None, min(Np, args.serve_saturated))):
        # None: every request queued at t = 0, the server's own capacity
        rate = frac * capacity if frac else float("inf")
        arrivals = serve.poisson_arrivals(count, rate, seed=5) if frac else None
        mism = []

        done = [0]

        def check(rep):
            if rep.error is None and serve.digest(rep.results) != ref[rep.rid]:
                mism.append(rep.rid)
            done[0] += 1
            if done[0] % 1000 == 0:
                log(f"served at {frac or 'saturation'}: {done[0]}/{count} replies")

        srv = serve.Server(cfg)
        replies = srv.run(pre[:count], arrivals, on_reply=check)
        ok = [r for r in replies if r.error is None]
        summ = serve.latency_summary(replies)
        run = {"requests": count, "rate_per_s": round(rate, 2) if frac else "all at t=0",
               "load": frac if frac else "saturated", **{k: round(v, 3) if isinstance(v, float)
                                                                else v for k, v in summ.items()},
               "by_size_decade": serve.latency_by_decade(replies),
               "graphs_per_s": len(ok) / srv.makespan, "makespan_s": round(srv.makespan, 3),
               "errors": len(replies) - len(ok), "mix_equals_alone": not mism, **srv.stats}
        log(f"served at {f'{frac}x capacity' if frac else 'saturation'}: {json.dumps(run)}")
        out["runs"].append(run)
        del replies
    out["resident"] = resident_run(pre[:200], cfg, capacity)
    del pre
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
    slow = sorted(hits, key=lambda r: -r.latency)[:10]
    last_build = max((r.arrival for r in builds), default=0.0)
    log("served, resident graphs: slowest queries (arrival after the last build's "
        "arrival in ms, latency in ms): "
        + ", ".join(f"({1e3 * (r.arrival - last_build):.0f}, {1e3 * r.latency:.1f})"
                    for r in slow))
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
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
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

    # Roofline of the dominant kernel, the count launch with the longest
    # device time (each count launch is timed on its own stream by HIP
    # events).  Algorithmic bytes per launch = the streamed candidates (4 B
    # each, 2 B for those read as 16-bit entries: pivots among the top 2^16
    # ranks) + 8 B per scanned pair (its in-pair word) + 8 B per pivot row.
    # The workgroup pivots among the top 2^16 ranks have a launch of their
    # own; the wavefront launches share the light bin's work statistics, so
    # when one of them dominates the light stage is priced as a whole.
    heavy16 = stages.get("count_heavy_bitmap16", 0.0)
    launches = {
        "count_heavy_bitmap16": heavy16,
        "count_heavy": stages["count_heavy"] - heavy16,
        "count_huge": stages["count_huge"],
        "count_light": max(stages.get("count_light_groups", 0.0), stages.get("count_light_wave", 0.0),
                           stages.get("count_light_bitmap", 0.0), 0.0)
        if work.get("algorithm") == 2 else stages["count_light"],
    }
    dom = max(launches, key=lambda k: launches[k])
    if dom == "count_heavy_bitmap16":
        c16 = work["cand_heavy_16"]
        algo_bytes = 2 * c16 + 8 * work["edges_heavy_16"] + 8 * work["rows_heavy_16"]
        dur_ms = heavy16
    else:
        b = {"count_light": "light", "count_heavy": "heavy", "count_huge": "huge"}[dom]
        c16 = work.get(f"cand_{b}_16", 0)
        e16 = work.get(f"edges_{b}_16", 0)
        r16 = work.get(f"rows_{b}_16", 0)
        if b == "heavy" and heavy16 > 0:  # the 16-bit pivots ran in their own launch
            algo_bytes = (4 * (work["cand_heavy"] - c16) + 8 * (work["edges_heavy"] - e16)
                          + 8 * (work["rows_heavy"] - r16))
            c16 = 0
        else:
            algo_bytes = (4 * (work[f"cand_{b}"] - c16) + 2 * c16 + 8 * work[f"edges_{b}"]
                          + 8 * work[f"rows_{b}"])
        dur_ms = stages[dom]
    dur_s = dur_ms / 1e3
    achieved = algo_bytes / dur_s / 1e9 if dur_s > 0 else 0.0
    digest = source_digest(COUNT_SOURCES)
    counters = counter_entry("count_heavy" if dom.startswith("count_heavy") else dom, digest) or {}
    kernel_names = {"count_light": "k_mid_groups + k_mid_wave + k_mid_block (light stage)",
                    "count_heavy": "k_mid_block (workgroup pivots: span bitmap / hash)",
                    "count_heavy_bitmap16": "k_mid_block (workgroup pivots among the top 2^16 "
                                            "ranks, 2048-word bitmap)",
                    "count_huge": "k_mid_block<LK_GLOBAL>"}
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
        "launch_ms": {k: round(v, 3) for k, v in launches.items()},
        "traffic_over_algorithmic": (round(counters["hbm_bytes_per_dispatch"] / algo_bytes, 3)
                                     if counters and algo_bytes else None),
        "avg_ms": round(dur_ms, 3),
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
                                                      "single_thread", "host_cpus", "cpu_model")}
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
