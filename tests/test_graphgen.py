"""The seeded generators: determinism, ranges and recipe sizes."""
import numpy as np

from paper_2105_00110_amd import graphgen as gg


def test_rmat_deterministic_and_thread_independent():
    a = gg.rmat(14, 16, seed=3, nthreads=1)
    b = gg.rmat(14, 16, seed=3, nthreads=7)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    c = gg.rmat(14, 16, seed=4)
    assert not np.array_equal(a[0], c[0])
    assert a[2] == 1 << 14 and a[0].shape[0] == 16 << 14
    assert a[0].min() >= 0 and a[0].max() < a[2]


def test_rmat_quadrant_frequencies():
    # without the scramble the top id bit is the first level's row choice,
    # which is 1 with probability c + d = 0.24
    src, dst, n = gg.rmat(10, 64, seed=9, scramble=False)
    top_row = (src >> 9) & 1
    top_col = (dst >> 9) & 1
    assert abs(top_row.mean() - 0.24) < 0.01
    assert abs(top_col.mean() - 0.24) < 0.01
    both = (top_row & top_col).mean()
    assert abs(both - 0.05) < 0.006


def test_scramble_is_a_bijection():
    src, dst, n = gg.rmat(12, 16, seed=5, scramble=False)
    s2, d2, _ = gg.rmat(12, 16, seed=5, scramble=True)
    # equal ids before the scramble stay equal after it, and only then
    order = np.argsort(src, kind="stable")
    a, b = src[order], s2[order]
    same_pre = a[1:] == a[:-1]
    same_post = b[1:] == b[:-1]
    np.testing.assert_array_equal(same_pre, same_post)


def test_er_edge_count():
    src, dst, n = gg.er(2000, 0.005, seed=1)
    expect = 0.005 * 2000 * 1999 / 2
    assert abs(len(src) - expect) < 5 * np.sqrt(expect)
    assert np.all(src < dst)
    src2, dst2, _ = gg.er(2000, 0.005, seed=1)
    np.testing.assert_array_equal(src, src2)


def test_ba_and_batched():
    src, dst, n = gg.ba(1000, 4, seed=2, cover=0.1)
    assert src.max() < n and dst.max() < n
    s, d, po, vo = gg.batched_ba(num_graphs=16, seed=8)
    ns, ms = gg.batched_ba_sizes(16, 8)
    assert po.shape == (17,) and vo[-1] == ns.sum()
    for g in range(16):
        a = s[po[g]:po[g + 1]]
        assert a.max() < ns[g]
    # the per-graph stream does not depend on the thread count
    s1, d1, _, _ = gg.batched_ba(num_graphs=16, seed=8, nthreads=1)
    np.testing.assert_array_equal(s, s1)
    gs, gd = gg.to_global(s, d, po, vo)
    assert gs.max() < vo[-1]
    ns_full, ms_full = gg.batched_ba_sizes()
    assert ns_full.min() >= 50 and ns_full.max() <= 20000
    assert ms_full.min() >= 2 and ms_full.max() <= 16
