"""Autotuner for the counting knobs of ``tc_tuning``.

The knobs (``include/tc.h``):

* ``algorithm``: wedge pivot (low or middle vertex of each triangle);
* ``light_max_dplus``: degree-bin threshold between wavefront rows and
  workgroup rows;
* ``item_pairs``: work-item tile, in (pivot, neighbour) pairs;
* ``heavy_block`` and ``light_block``: workgroup shapes;
* ``lds_max_entries``: largest LDS table;
* ``bitmap_words``: LDS bitmap size for workgroup pivots (0 = hash only);
* ``light_bitmap_pairs``: pair count from which wavefront pivots move to the
  bitmap kernel (0 = never).

``tune_fused`` searches the knobs of the fused batch launch
(``tc_fused_tuning``: workgroup size, workgroups per compute unit) and the
order in which graphs are taken from its queue (largest first or as given)
by exhaustive search, each trial timed by HIP events and compared bit for
bit with the first.

``tune`` runs a coordinate search on a built graph.  It starts from the
library defaults (or a given start) and sweeps one knob at a time over its
candidate values, keeping a value only when the measured device time of the
counting stages drops.  Every trial's results are compared bit for bit with
the first trial's, and a mismatch raises.  The best settings are stored per
workload class in a JSON file that ``bench.py`` and the serving loop read.
"""
import json
import os
import time

from . import tc

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_FILE = os.path.join(HERE, "tuning", "mi355x.json")

SPACE = {
    "algorithm": [tc.TC_ALGO_LOW_PIVOT, tc.TC_ALGO_MID_PIVOT],
    "light_max_dplus": [32, 64, 128, 256, 512, 1024],
    "item_pairs": [128, 256, 512, 1024, 2048, 4096],
    "heavy_block": [256, 512, 1024],
    "light_block": [128, 256, 512],
    "lds_max_entries": [2048, 4096, 8192],
    "bitmap_words": [0, 1024, 2048, 4096, 8192],
    "light_bitmap_pairs": [0, 16, 64, 256, 1024],
}

# stages that the counting knobs change
TUNED_STAGES = ("bin", "count_light", "count_heavy", "count_huge", "fold")


def default_tuning():
    t = tc.tc_tuning_default()
    return {k: int(getattr(t, k)) for k, _ in t._fields_}


def _results_device(g):
    r = g.results_device()
    return {k: v.clone() for k, v in r.items()}


def _same(a, b):
    import torch
    return all(torch.equal(a[k], b[k]) for k in a)


def measure(g, tuning, reps=2):
    """Median over reps of the summed device time (ms) of the tuned stages."""
    times = []
    for _ in range(reps):
        g.compute(tuning)
        ms = g.stage_ms()
        times.append(sum(ms[k] for k in TUNED_STAGES))
    times.sort()
    return times[len(times) // 2]


def tune(g, space=None, start=None, reps=2, rounds=2, budget_s=120.0, log=None):
    """Coordinate search on graph g (a built ``tc.Graph``).

    Returns ``{"tuning", "ms", "default_ms", "trials"}``.
    """
    space = space or SPACE
    tc.tc_set_profiling(True)
    cur = dict(start or default_tuning())
    g.compute(cur)
    ref = _results_device(g)
    best_ms = measure(g, cur, reps)
    default_ms = best_ms
    trials = [{"tuning": dict(cur), "ms": round(best_ms, 3)}]
    t0 = time.perf_counter()
    for _ in range(rounds):
        improved = False
        for knob, values in space.items():
            for v in values:
                if v == cur[knob] or time.perf_counter() - t0 > budget_s:
                    continue
                cand = dict(cur, **{knob: v})
                try:
                    ms = measure(g, cand, reps)
                except tc.TCError as e:  # knob combination the library rejects
                    trials.append({"tuning": cand, "error": str(e)})
                    continue
                if not _same(_results_device(g), ref):
                    raise RuntimeError(f"tuning {cand} changed the results")
                trials.append({"tuning": cand, "ms": round(ms, 3)})
                if log:
                    log(f"autotune {knob}={v}: {ms:.3f} ms (best {best_ms:.3f})")
                if ms < best_ms * 0.99:
                    best_ms, cur, improved = ms, cand, True
        if not improved:
            break
    return {"tuning": cur, "ms": round(best_ms, 3), "default_ms": round(default_ms, 3),
            "trials": trials}


def load(workload, path=DEFAULT_FILE):
    """Stored tuning for a workload class, or None."""
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    w = d.get("workloads", {}).get(workload)
    return dict(w["tuning"]) if w else None


def store(workload, result, path=DEFAULT_FILE, device=None):
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        d = {}
    d.setdefault("workloads", {})
    if device:
        d["device"] = device
    d["workloads"][workload] = {k: result[k] for k in ("tuning", "ms", "default_ms")}
    d["workloads"][workload]["trials"] = len(result["trials"])
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


FUSED_SPACE = {"block": [256, 512, 1024], "wg_per_cu": [1, 2, 4], "order": ["largest_first", None]}


def _fused_outputs(fb):
    """Per-graph outputs of a FusedBatch run (the rows past m_g are not
    outputs and are left out)."""
    res = fb.results()
    return [fb.graph(res, g) for g in range(fb.G)]


def _fused_same(a, b):
    import numpy as np
    for x, y in zip(a, b):
        for k in ("eu", "ev", "support", "tri", "num", "triG"):
            if not np.array_equal(x[k], y[k]):
                return False
        if not np.array_equal(x["tc"].view(np.uint64), y["tc"].view(np.uint64)) or \
                x["status"] != y["status"]:
            return False
    return True


def tune_fused(src, dst, pair_off, vtx_off, space=None, reps=3, log=None):
    """Exhaustive search over the fused launch's knobs for one batch.

    ``src``/``dst`` are device tensors, the offsets host arrays.  Returns
    ``{"tuning", "ms", "default_ms", "trials"}`` with ``tuning`` holding
    block, wg_per_cu and order."""
    import itertools

    import torch
    space = space or FUSED_SPACE
    trials, ref, best, default_ms = [], None, None, None
    d = tc.tc_fused_tuning_default().as_dict()
    combos = [dict(zip(space, c)) for c in itertools.product(*space.values())]
    combos.sort(key=lambda c: (c["block"], c["wg_per_cu"]) != (d["block"], d["wg_per_cu"]) or
                c["order"] != "largest_first")  # the default first
    for c in combos:
        fb = tc.FusedBatch(src, dst, pair_off, vtx_off, order=c["order"],
                           tuning={"block": c["block"], "wg_per_cu": c["wg_per_cu"]})
        fb.run()
        torch.cuda.synchronize()
        out = _fused_outputs(fb)
        if ref is None:
            ref = out
        elif not _fused_same(out, ref):
            raise RuntimeError(f"fused tuning {c} changed the results")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(reps):
            e0.record()
            fb.run()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = sorted(times)[len(times) // 2]
        if default_ms is None:
            default_ms = ms
        trials.append({"tuning": c, "ms": round(ms, 3)})
        if log:
            log(f"autotune fused {c}: {ms:.3f} ms")
        if best is None or ms < best[1]:
            best = (c, ms)
        del fb
    return {"tuning": best[0], "ms": round(best[1], 3), "default_ms": round(default_ms, 3),
            "trials": trials}
