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
    b = ctypes.c_int64(0)
    assert lib.tc_compute_bytes(None, None, None, ctypes.byref(b)) == tc.TC_ERR_INVALID_ARG
    assert lib.tc_set_memory_limit(-1) == tc.TC_ERR_INVALID_ARG
    assert lib.tc_set_memory_limit(0) == tc.TC_OK


def test_fused_argument_checks_on_host():
    # argument errors are found before any device work
    lib = tc.load()
    ft = tc.tc_fused_tuning_default()
    assert ft.block in (256, 512, 1024) and 1 <= ft.wg_per_cu <= 16
    assert tc.tc_batch_fused_workspace_bytes(-1, 0, 0) == -1
    ws = tc.tc_batch_fused_workspace_bytes(1000, 100, 3)
    assert ws >= 20 * 1000 + 40 * 100
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below fails its checks
    args = [fake, fake, fake, fake, None, 3, 1000, 100] + [fake] * 9
    assert lib.tc_batch_fused(*args, fake, ws - 1, None, None) == tc.TC_ERR_INVALID_ARG
    assert lib.tc_batch_fused(*args, ctypes.c_void_p((1 << 20) + 8), ws, None,
                              None) == tc.TC_ERR_INVALID_ARG
    bad = tc.tc_fused_tuning(block=384, wg_per_cu=2)
    assert lib.tc_batch_fused(*args, fake, ws, ctypes.byref(bad), None) == tc.TC_ERR_INVALID_ARG
    neg = [fake, fake, fake, fake, None, -1, 1000, 100] + [fake] * 9
    assert lib.tc_batch_fused(*neg, fake, ws, None, None) == tc.TC_ERR_INVALID_ARG
    none_status = args[:16] + [None]
    assert lib.tc_batch_fused(*none_status, fake, ws, None, None) == tc.TC_ERR_INVALID_ARG
    # no graphs: nothing to do, nothing touched
    empty = [None, None, None, None, None, 0, 0, 0] + [None] * 9
    assert lib.tc_batch_fused(*empty, None, 0, None, None) == tc.TC_OK


def test_no_oracle_in_product():
    pkg = os.path.join(ROOT, "paper_2105_00110_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".c", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt, f
