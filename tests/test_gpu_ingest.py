"""GPU: order-preserving relabelling of arbitrary ids, and graphs read from
text files end to end (libtc through its C ABI, against numpy for the
relabel and against the oracle for the results)."""
import numpy as np
import pytest

from oracle import native
from paper_2105_00110_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


def _np_relabel(src, dst):
    ids = np.unique(np.concatenate([src, dst]))
    return (np.searchsorted(ids, src).astype(np.int32), np.searchsorted(ids, dst).astype(np.int32),
            ids)


@pytest.mark.parametrize("P, span, seed", [(1, 10, 1), (1000, 50, 2), (200000, 1 << 62, 3),
                                           (100000, 1 << 20, 4)])
def test_relabel_matches_numpy(tclib, P, span, seed):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, span, P, dtype=np.int64)
    dst = rng.integers(0, span, P, dtype=np.int64)
    _say("relabel", P, span)
    s32, d32, ids, n = tclib.relabel(src, dst)
    es, ed, eids = _np_relabel(src, dst)
    assert n == len(eids)
    np.testing.assert_array_equal(ids, eids)
    np.testing.assert_array_equal(s32, es)
    np.testing.assert_array_equal(d32, ed)


def test_relabel_device_memory(tclib):
    rng = np.random.default_rng(9)
    src = rng.integers(0, 1 << 40, 5000, dtype=np.int64)
    dst = rng.integers(0, 1 << 40, 5000, dtype=np.int64)
    ds, dd = torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda()
    s32 = torch.empty(5000, dtype=torch.int32, device="cuda")
    d32 = torch.empty_like(s32)
    ids = torch.empty(10000, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    n = tclib.tc_relabel_ids(ds.data_ptr(), dd.data_ptr(), 5000, s32.data_ptr(), d32.data_ptr(),
                             ids.data_ptr(), tclib.TC_MEM_DEVICE, stream)
    es, ed, eids = _np_relabel(src, dst)
    assert n == len(eids)
    np.testing.assert_array_equal(s32.cpu().numpy(), es)
    np.testing.assert_array_equal(d32.cpu().numpy(), ed)
    np.testing.assert_array_equal(ids[:n].cpu().numpy(), eids)


def test_relabel_rejects_negative(tclib):
    with pytest.raises(tclib.TCError):
        tclib.relabel(np.array([1, -5], np.int64), np.array([2, 3], np.int64))


@pytest.mark.parametrize("family", ["rmat_s13", "ba_3000", "fig_bridge"])
def test_text_file_end_to_end(tclib, tmp_path, family):
    if family == "rmat_s13":
        s, d, n = gg.rmat(13, 16, seed=13)
    elif family == "ba_3000":
        s, d, n = gg.ba(3000, 5, seed=8)
    else:
        s, d, n = gg.bridge_cliques(5, 6)
    su, du = gg.sparse_ids(s), gg.sparse_ids(d)
    path = str(tmp_path / "g.txt")
    gg.write_text(path, su, du)
    _say("text file", family, len(s), "pairs")
    g, ids = tclib.Graph.from_text(path)
    g.compute()
    res = g.results()
    eu, ev = g.edges()
    g.close()
    # the oracle on the same graph, relabelled by numpy
    rs, rd, eids = _np_relabel(su, du)
    np.testing.assert_array_equal(ids, eids)
    ref = native.o2_paper(rs, rd, len(eids))
    np.testing.assert_array_equal(eu, ref.eu)
    np.testing.assert_array_equal(ev, ref.ev)
    np.testing.assert_array_equal(res["support"], ref.sup)
    np.testing.assert_array_equal(res["tri"], ref.tri)
    np.testing.assert_array_equal(res["num"], ref.num)
    np.testing.assert_array_equal(res["tc"].view(np.uint64), ref.tc.view(np.uint64))
    assert int(res["triG"][0]) == ref.triG
