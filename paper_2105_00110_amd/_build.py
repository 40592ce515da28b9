"""In-tree build of the native libraries.

* ``gen/libtcgen.so``   -- seeded input generators (host C, gcc).
* ``libtc.so``          -- the HIP library behind ``include/tc.h``
                           (hipcc, gfx950 only).

Both are rebuilt on every call; the .so files are written next to the
sources so that they travel with the source tree.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
GEN_SRC = os.path.join(HERE, "gen", "graphgen.c")
GEN_LIB = os.path.join(HERE, "gen", "libtcgen.so")
TC_LIB = os.path.join(HERE, "libtc.so")
OBJ_DIR = os.path.join(ROOT, "_build", "obj")

HIP_SOURCES = [
    "tc_sort.hip",
    "tc_scan.hip",
    "tc_build.hip",
    "tc_count.hip",
    "tc_count_mid.hip",
    "tc_aggregate.hip",
    "tc_algebraic.hip",
    "tc_ingest.hip",
    "tc_fused.hip",
    "tc_api.hip",
]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    # no packed-fp32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off",
    "-fno-fast-math",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build_gen(verbose=False):
    tmp = GEN_LIB + ".tmp"
    _run(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-o", tmp,
          GEN_SRC, "-lm"], verbose)
    os.replace(tmp, GEN_LIB)
    return GEN_LIB


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build_hip(verbose=False, jobs=None):
    os.makedirs(OBJ_DIR, exist_ok=True)
    cc = hipcc()
    objs = []
    cmds = []
    for s in HIP_SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(OBJ_DIR, s.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([cc, *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj])
    jobs = jobs or min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = TC_LIB + ".tmp"
    _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, TC_LIB)
    return TC_LIB


def build(verbose=False):
    build_gen(verbose)
    build_hip(verbose)


if __name__ == "__main__":
    build(verbose=True)
