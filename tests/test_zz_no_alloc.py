"""GPU: tc_batch_fused_noalloc (the fused batch with the library's fixed
device workspace) against tc_batch_fused (caller workspace) through the C
ABI: two calls in a row, the second with a smaller batch, each output equal
to the workspace entry point's; a batch whose workspace exceeds the fixed
array is refused before any work."""
import numpy as np
import pytest

from paper_2105_00110_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


def _batch(graphs):
    src = np.concatenate([np.asarray(g[0], np.int32) for g in graphs])
    dst = np.concatenate([np.asarray(g[1], np.int32) for g in graphs])
    po = np.zeros(len(graphs) + 1, np.int64)
    vo = np.zeros(len(graphs) + 1, np.int64)
    np.cumsum([len(g[0]) for g in graphs], out=po[1:])
    np.cumsum([g[2] for g in graphs], out=vo[1:])
    return src, dst, po, vo


def _noalloc(tc, fb):
    """Runs tc_batch_fused_noalloc on fb's inputs into fresh outputs (filled
    with marker values first); returns them as host arrays."""
    dev = fb.src.device
    P1, N1, G1 = max(fb.P, 1), max(fb.N, 1), max(fb.G, 1)
    out = {"eu": torch.full((P1,), -5, dtype=torch.int32, device=dev),
           "ev": torch.full((P1,), -5, dtype=torch.int32, device=dev),
           "support": torch.full((P1,), -5, dtype=torch.int64, device=dev),
           "num_edges": torch.full((G1,), -5, dtype=torch.int64, device=dev),
           "tri": torch.full((N1,), -5, dtype=torch.int64, device=dev),
           "triG": torch.full((G1,), -5, dtype=torch.int64, device=dev),
           "num": torch.full((N1,), -5, dtype=torch.int64, device=dev),
           "tc": torch.full((N1,), -5.0, dtype=torch.float64, device=dev),
           "status": torch.full((G1,), 99, dtype=torch.int32, device=dev)}
    torch.cuda.synchronize()
    p = lambda t: t.data_ptr()
    st = tc.tc_batch_fused_noalloc(p(fb.src), p(fb.dst), p(fb.pair_off), p(fb.vtx_off),
                                   p(fb.order), fb.G, fb.P, fb.N, p(out["eu"]), p(out["ev"]),
                                   p(out["support"]), p(out["num_edges"]), p(out["tri"]),
                                   p(out["triG"]), p(out["num"]), p(out["tc"]), p(out["status"]),
                                   None, fb.stream)
    assert st == 0
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    for k in ("support", "tri", "triG", "num"):
        res[k] = res[k].view(np.uint64)
    return res


def test_noalloc_equals_workspace_entry_point_twice(tclib):
    big = ([gg.er(2000, 0.005, seed=s) for s in range(1, 6)] + [gg.ba(3000, 8, seed=3)]
           + [gg.rmat(14, 16, seed=5), gg.clique(200)])
    small = [gg.er(2000, 0.005, seed=7), gg.clique(12)]
    for name, graphs in (("larger", big), ("smaller", small)):
        src, dst, po, vo = _batch(graphs)
        need = tclib.tc_batch_fused_workspace_bytes(int(po[-1]), int(vo[-1]), len(graphs))
        _say("no-alloc call,", name, "batch:", len(graphs), "graphs,", int(po[-1]), "pairs,",
             need, "workspace bytes")
        assert need <= tclib.tc_batch_fused_noalloc_max_bytes()
        fb = tclib.FusedBatch(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(), po, vo)
        fb.run()
        torch.cuda.synchronize()
        ref = fb.results()
        got = _noalloc(tclib, fb)
        for k in ("num_edges", "tri", "triG", "num", "status"):
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
        np.testing.assert_array_equal(got["tc"].view(np.uint64), ref["tc"].view(np.uint64))
        assert np.all(ref["status"] >= 0)
        for g in range(len(graphs)):
            a, b = fb.graph(got, g), fb.graph(ref, g)
            for k in ("eu", "ev", "support"):
                np.testing.assert_array_equal(a[k], b[k], err_msg=f"{k} graph {g}")


def test_noalloc_refuses_batches_beyond_its_array(tclib):
    # a batch whose workspace would not fit: refused on the host, nothing queued
    import ctypes
    lib = tclib.load()
    cap = tclib.tc_batch_fused_noalloc_max_bytes()
    P = cap // 20 + 1
    assert tclib.tc_batch_fused_workspace_bytes(P, 1, 1) > cap
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: the call stops at the size check
    st = lib.tc_batch_fused_noalloc(fake, fake, fake, fake, None, 1, P, 1,
                                    *([fake] * 9), None, None)
    assert st == tclib.TC_ERR_BUDGET
