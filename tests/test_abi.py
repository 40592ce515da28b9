"""CPU-side checks of the C ABI: the library loads and exports every entry
point include/tc.h declares (no compute call: no GPU here)."""
import ctypes
import os
import re

from paper_2105_00110_amd import tc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "tc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = tc.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    for name in declared_functions():
        assert name in tc._SIGS, name
        assert callable(getattr(tc, name)), name


def test_host_only_calls():
    assert tc.tc_version() == 10000
    assert tc.tc_status_string(tc.TC_ERR_VERTEX_RANGE).startswith("vertex id")
    t = tc.tc_tuning_default()
    assert t.light_max_dplus >= 2 and t.heavy_block % 64 == 0
    assert tc.tc_estimate_device_bytes(1000, 100) > 0
    assert tc.tc_estimate_device_bytes(-1, 100) == -1
    lib = tc.load()
    assert lib.tc_num_vertices(None) == -1
    assert lib.tc_num_edges(None) == -1
    lib.tc_graph_destroy(None)
    h = ctypes.c_void_p()
    assert lib.tc_graph_from_edges(None, None, -1, 5, 0, None, ctypes.byref(h)) == tc.TC_ERR_INVALID_ARG
    assert lib.tc_graph_from_edges(None, None, 0, 5, 7, None, ctypes.byref(h)) == tc.TC_ERR_INVALID_ARG
    assert lib.tc_numerator_algebraic(None, None, 0, None) == tc.TC_ERR_INVALID_ARG


def test_no_oracle_in_product():
    pkg = os.path.join(ROOT, "paper_2105_00110_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".c", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt, f
