"""Host logic of bench.py: the counter summary's byte rule and kernel
matching, on synthetic rocprofv3 CSVs (no GPU)."""
import csv
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


COPY = "__amd_rocclr_copyBuffer"
MID = "void (anonymous namespace)::k_mid_block<2>(int, unsigned int const*)"
MID16 = "(anonymous namespace)::k_mid_block16(int, unsigned int const*)"


def test_counter_summary_rule_and_shapes(tmp_path):
    b = _bench()
    d = tmp_path / "pmc"
    # dispatches: the light bitmap launch (grid 100) and the top-2^16
    # workgroup launch (grid 200), in two steps; then the 1 GiB copy (three
    # dispatches)
    disp = [(COPY, 4096, 0), (MID, 100, 1), (MID16, 200, 2), (MID, 100, 3), (MID16, 200, 4),
            (COPY, 4096, 5), (COPY, 4096, 6), (COPY, 4096, 7)]
    p1, p2 = [], []
    for name, grid, i in disp:
        copy = name == COPY and i > 0  # dispatch 0: a small copy of the same shape
        c1 = {"TCC_EA0_RDREQ_sum": 8388608 if copy else 1000 + grid,
              "TCC_EA0_RDREQ_32B_sum": 0 if copy else 10,
              "TCC_EA0_RDREQ_64B_sum": 0 if copy else 20,
              "TCC_EA0_RDREQ_128B_sum": 8388608 if copy else 1000 + grid - 30,
              "SQ_ACTIVE_INST_VALU": 50, "SQ_INSTS_VALU": 400, "SQ_WAVES": 64,
              "GRBM_GUI_ACTIVE": 800}
        c2 = {"TCC_EA0_WRREQ_sum": 16777216 if copy else 300,
              "TCC_EA0_WRREQ_64B_sum": 16777216 if copy else 100,
              "TCC_HIT_sum": 1, "TCC_MISS_sum": 3, "SQ_INSTS_LDS": 5,
              "SQ_LDS_BANK_CONFLICT": 2, "SQ_ACTIVE_INST_LDS": 4, "SQ_INSTS_VMEM_RD": 7}
        for rows, c in ((p1, c1), (p2, c2)):
            for k, v in c.items():
                rows.append({"Dispatch_Id": i, "Grid_Size": grid, "Kernel_Name": name,
                             "Counter_Name": k, "Counter_Value": v})
    p3 = []
    for name, grid, i in disp:
        copy = name == COPY and i > 0
        c3 = {"TCC_EA0_RDREQ_DRAM_sum": 8388608 if copy else 600,
              "TCC_EA0_WRREQ_DRAM_sum": 16777216 if copy else 300,
              "TCC_EA0_RDREQ_sum": 8388608 if copy else 1000 + grid,
              "TCC_EA0_WRREQ_sum": 16777216 if copy else 300}
        for k, v in c3.items():
            p3.append({"Dispatch_Id": i, "Grid_Size": grid, "Kernel_Name": name,
                       "Counter_Name": k, "Counter_Value": v})
    _write(str(d / "pmc_1" / "host" / "run_counter_collection.csv"), p1)
    _write(str(d / "pmc_2" / "host" / "run_counter_collection.csv"), p2)
    _write(str(d / "pmc_3" / "host" / "run_counter_collection.csv"), p3)
    trace = [{"Kernel_Name": name, "Grid_Size_X": grid, "Grid_Size_Y": 1, "Grid_Size_Z": 1,
              "Start_Timestamp": 0, "End_Timestamp": (3_000_000 if grid == 200 else 1_000_000)}
             for name, grid, _ in disp]
    _write(str(d / "ktrace" / "host" / "run_kernel_trace.csv"), trace)
    _write(str(d / "ktrace" / "host" / "run_kernel_stats.csv"),
           [{"Name": MID, "AverageNs": 1_000_000}, {"Name": MID16, "AverageNs": 3_000_000},
            {"Name": COPY, "AverageNs": 400_000}])
    b.summarize_counters(str(d), out_dir=str(tmp_path))
    out = json.load(open(tmp_path / "counters_rmat_s24.json"))
    k = out["kernels"]
    assert out["copy_check"]["read_ratio"] == 1.0 and out["copy_check"]["write_ratio"] == 1.0
    assert k["count_heavy"]["kernel"] == "k_mid_block16"
    assert k["count_light_bitmap"]["kernel"] == "k_mid_block<2>"
    assert k["count_heavy"]["avg_ms"] == 3.0 and k["count_light_bitmap"]["avg_ms"] == 1.0
    # 32 B x 10 + 64 B x 20 + 128 B x the rest; 64 B x 100 + 32 B x 200
    h = k["count_heavy"]
    assert h["hbm_read_bytes"] == 32 * 10 + 64 * 20 + 128 * (1200 - 30)
    assert h["hbm_write_bytes"] == 64 * 100 + 32 * 200
    assert h["hbm_bytes_per_dispatch"] == h["hbm_read_bytes"] + h["hbm_write_bytes"]
    assert h["dispatches"] == 2 and h["rdreq_unsized"] == 0
    assert h["rdreq_dram_fraction"] == 0.5 and h["wrreq_dram_fraction"] == 1.0
    assert out["source_digest"] == b.source_digest(b.COUNT_SOURCES)
    assert os.path.exists(tmp_path / "counters_rmat_s24.md")


def test_counter_entry_only_for_the_current_source(tmp_path, monkeypatch):
    b = _bench()
    assert b.counter_entry("no_such_kernel", "0") is None
