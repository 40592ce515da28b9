"""Text edge-list reader (host code of libtc; no GPU)."""
import numpy as np
import pytest

from paper_2105_00110_amd import graphgen as gg
from paper_2105_00110_amd import tc


def _write(tmp_path, text, name="g.txt"):
    p = tmp_path / name
    p.write_bytes(text.encode())
    return str(p)


def test_formats_comments_columns_crlf(tmp_path):
    text = ("# SNAP-style header\n% another comment\n\n"
            "1 2\n"
            "3\t4\n"
            "  5   6  \n"
            "7 8 1.5 extra\n"
            "9 10\r\n"
            "18446744073 9223372036854775807\n"
            "11 12")  # no final newline
    src, dst = tc.read_edge_text(_write(tmp_path, text))
    np.testing.assert_array_equal(src, [1, 3, 5, 7, 9, 18446744073, 11])
    np.testing.assert_array_equal(dst, [2, 4, 6, 8, 10, 9223372036854775807, 12])


@pytest.mark.parametrize("bad, line", [("1 2\n3\n", 2), ("1 2\n# c\n-1 4\n", 3),
                                       ("1 2\n3 x\n", 2), ("1 2\n3 9223372036854775808\n", 2),
                                       ("1,2\n", 1)])
def test_malformed_lines_named(tmp_path, bad, line):
    with pytest.raises(tc.TCError, match=f"malformed line {line}"):
        tc.read_edge_text(_write(tmp_path, bad))


def test_missing_file_and_empty(tmp_path):
    st, P, _ = tc.tc_edge_text_read(str(tmp_path / "nope.txt"))
    assert st == tc.TC_ERR_IO and P == 0
    src, dst = tc.read_edge_text(_write(tmp_path, ""))
    assert src.size == 0 and dst.size == 0
    src, dst = tc.read_edge_text(_write(tmp_path, "# only comments\n\n", "c.txt"))
    assert src.size == 0


def test_capacity_too_small(tmp_path):
    p = _write(tmp_path, "1 2\n3 4\n5 6\n")
    a = np.empty(2, np.int64)
    b = np.empty(2, np.int64)
    st, P, _ = tc.tc_edge_text_read(p, a, b, 2)
    assert st == tc.TC_ERR_INVALID_ARG and P == 3


@pytest.mark.parametrize("threads", [1, 3, 8, 64])
def test_chunking_matches_python_parse(tmp_path, threads):
    s, d, n = gg.rmat(12, 16, seed=4)
    su, du = gg.sparse_ids(s), gg.sparse_ids(d)
    p = str(tmp_path / "r.txt")
    gg.write_text(p, su, du)
    src, dst = tc.read_edge_text(p, nthreads=threads)
    np.testing.assert_array_equal(src, su)
    np.testing.assert_array_equal(dst, du)
    # an independent parse of the same file
    rows = [ln.split() for ln in open(p) if ln.strip() and not ln.startswith("#")]
    np.testing.assert_array_equal(src, np.array([int(r[0]) for r in rows], np.int64))
    np.testing.assert_array_equal(dst, np.array([int(r[1]) for r in rows], np.int64))


def test_sparse_ids_order_preserving():
    x = np.arange(5000, dtype=np.int64)
    y = gg.sparse_ids(x, seed=3)
    assert np.all(np.diff(y) > 0) and y.min() >= (1 << 40)
