"""Kernels of the middle-pivot count (tc_count_mid.hip), compiled for the
host with a CPU emulation of the device features they use
(tests/emu/hip_cpu.h: one thread per lane, wavefront and workgroup
barriers), against brute force.

Folds: k_fold and k_fold_big run on random triangular bit matrices against
brute-force row and column counts.

The fold turns each row u's bit matrix B_u into supports: row i's popcount
counts the triangles on (u, N_H(u)[i]) as (low, middle) edge, column j's sum
those on (u, N_H(u)[j]) as (low, high) edge (the support updates of
Procedure 1 that lie in u's row).  Covered: the byte-counter butterfly of
rows of 2..64 entries, the 16-bit SWAR flush and private partials of rows
up to 1024 entries, the one-owner and atomic adds of longer rows, the
64-bit-offset kernel, rows above the LDS counter cap, all-ones matrices
(the largest counts), and the aligned 16-byte row-sum loads, under
AddressSanitizer (a read past the 4 words of padding that follow the last
row fails the test).

Probe of the pivots among the top 2^16 ranks: bitmap_build (an emulated
workgroup) against the bitmap's definition, and bitmap16_run on random
runs of a 16-bit column stream (odd and even starts, full and partial
runs, values outside the row and below the 16-bit base) against the hit
masks and per-place counts that brute force gives.  Host code only: no
GPU."""
import pathlib
import re
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
SRC = ROOT / "paper_2105_00110_amd" / "csrc" / "tc_count_mid.hip"
EMU = ROOT / "tests" / "emu"


def _segment(src, start, end):
    i = src.index(start)
    return src[i:src.index(end, i)]


def fold_body(src):
    """The fold kernels and the helpers they use, as host code."""
    parts = [
        _segment(src, "// Words of the bit rows of a row with d entries", "static inline unsigned grid_for"),
        _segment(src, "__device__ __forceinline__ void planes_flush(", "__global__ void k_dplus_flags"),
    ]
    body = "\n".join(parts)
    dyn = "extern __shared__ uint32_t colc_all[];"
    assert dyn in body
    body = body.replace(dyn, "uint32_t *colc_all = colc_lds;")
    return "static uint32_t *colc_lds;  // the launch's dynamic LDS\n" + body


def probe16_body(src):
    """bitmap_build and bitmap16_run, as host code."""
    return "\n".join([
        _segment(src, "// Builds the bitmap of row ocol", "// One lane's 32-entry run of a pair's tail"),
        _segment(src, "// One lane's 32-entry run of a pair's tail", "// ----"),
    ])


def _build_and_run(tmp_path, name, body_name, body):
    (tmp_path / body_name).write_text(body)
    exe = tmp_path / name
    cmd = ["g++", "-std=c++20", "-O1", "-pthread", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-Wno-unused-function", f"-I{EMU}", f"-I{tmp_path}", str(EMU / f"{name}.cpp"),
           str(EMU / "emu_rt.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_fold_kernels_on_cpu_emulation(tmp_path):
    out = _build_and_run(tmp_path, "fold_check", "fold_body.inc", fold_body(SRC.read_text()))
    lines = [l for l in out.splitlines() if "mismatches" in l]
    assert len(lines) == 4
    assert all(re.search(r", 0 mismatches$", l) for l in lines), lines


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_top_16_bit_probe_on_cpu_emulation(tmp_path):
    out = _build_and_run(tmp_path, "probe16_check", "probe16_body.inc",
                         probe16_body(SRC.read_text()))
    lines = [l for l in out.splitlines() if l.startswith("row of")]
    assert len(lines) == 6
    assert all(re.search(r"bitmap mismatches 0; \d+ runs, mask mismatches 0, count mismatches 0$", l)
               for l in lines), lines
