"""Graphs on disk, host side (no GPU): the CSR file the library writes and
reads, the split into vertex ranges of at most part_edges edges (a longer row
alone), 64-bit edge offsets beyond 2^31, malformed files, and the argument
checks of trw_disk_walk that run before any device work."""
import ctypes
import os

import numpy as np
import pytest

import synth

trw = pytest.importorskip("paper_2107_11983_amd")
from paper_2107_11983_amd import _abi  # noqa: E402


def greedy_ranges(row_ptr, part_edges):
    """Vertex ranges, each as long as its edges stay within part_edges (the first row
    of a range is always taken): the split the open call documents."""
    n = len(row_ptr) - 1
    out, v = [], 0
    while v < n:
        v0, e0 = v, row_ptr[v]
        v += 1
        while v < n and row_ptr[v + 1] - e0 <= part_edges:
            v += 1
        out.append((v0, v, int(row_ptr[v0]), int(row_ptr[v])))
    return out


def small_graph():
    g = synth.rmat(10, 8, False, 77)
    synth.attach_attrs(g, 78, weights=True, labels=4)
    return g


def test_write_then_read_back(tmp_path):
    g = small_graph()
    path = str(tmp_path / "g.csr")
    trw.write_disk_graph(path, g.row_ptr.astype(np.int64), g.col, g.weight, g.label)
    n, m = g.n, g.m
    raw = np.fromfile(path, np.uint8)
    assert raw[:8].tobytes() == b"TRWCSR1\0"
    head = raw[8:32].view(np.uint64)
    assert list(head) == [n, m, 3]
    o = 32
    assert np.array_equal(raw[o:o + 8 * (n + 1)].view(np.int64), g.row_ptr)
    o += 8 * (n + 1)
    assert np.array_equal(raw[o:o + 4 * m].view(np.int32), g.col)
    o += 4 * m
    assert np.array_equal(raw[o:o + 4 * m].view(np.uint32), g.weight)
    o += 4 * m
    assert np.array_equal(raw[o:o + m], g.label)
    assert raw.size == o + m
    G = trw.DiskGraph(path, 0)
    assert (G.n, G.m, G.flags, G.parts) == (n, m, 3, 1)
    assert G.partition(0) == (0, n, 0, m)
    G.close()


@pytest.mark.parametrize("part_edges", [1, 7, 100, 1000, 4095])
def test_partitions_follow_the_rule(tmp_path, part_edges):
    g = small_graph()
    path = str(tmp_path / "g.csr")
    trw.write_disk_graph(path, g.row_ptr, g.col, g.weight)
    G = trw.DiskGraph(path, part_edges)
    want = greedy_ranges(g.row_ptr.astype(np.int64), part_edges)
    assert G.parts == len(want)
    got = [G.partition(i) for i in range(G.parts)]
    assert got == want
    # they tile the vertices; each holds at most part_edges edges unless it is one row
    assert got[0][0] == 0 and got[-1][1] == g.n
    for (a, b, c, d), nxt in zip(got, got[1:] + [None]):
        assert d - c <= part_edges or b - a == 1
        if nxt:
            assert nxt[0] == b
    with pytest.raises(trw.TrwError):
        G.partition(G.parts)
    G.close()


def test_empty_rows_and_no_edges(tmp_path):
    path = str(tmp_path / "e.csr")
    trw.write_disk_graph(path, np.zeros(6, np.int64), np.zeros(0, np.int32))
    G = trw.DiskGraph(path, 3)
    assert (G.n, G.m, G.parts) == (5, 0, 1)
    assert G.partition(0) == (0, 5, 0, 0)
    G.close()


def test_edge_offsets_beyond_2_31(tmp_path):
    """A sparse file with m = 2^31 + 10: rows of 2^30 edges, then short ones.  Only the
    header and row_ptr are read at open, so the partition bounds are checked without
    touching the edges."""
    n = 4
    rp = np.array([0, 1 << 30, 1 << 31, (1 << 31) + 5, (1 << 31) + 10], np.int64)
    m = int(rp[-1])
    path = str(tmp_path / "big.csr")
    with open(path, "wb") as f:
        f.write(b"TRWCSR1\0")
        f.write(np.array([n, m, 0], np.uint64).tobytes())
        f.write(rp.tobytes())
        f.truncate(32 + 8 * (n + 1) + 4 * m)
    G = trw.DiskGraph(path, 1 << 30)
    assert (G.n, G.m, G.parts) == (n, m, 3)
    assert [G.partition(i) for i in range(3)] == [(0, 1, 0, 1 << 30), (1, 2, 1 << 30, 1 << 31),
                                                  (2, 4, 1 << 31, (1 << 31) + 10)]
    G.close()
    # a row of 2^31 edges cannot be one partition: refused
    rp2 = np.array([0, 1 << 31, (1 << 31) + 1], np.int64)
    path2 = str(tmp_path / "row.csr")
    with open(path2, "wb") as f:
        f.write(b"TRWCSR1\0")
        f.write(np.array([2, int(rp2[-1]), 0], np.uint64).tobytes())
        f.write(rp2.tobytes())
        f.truncate(32 + 8 * 3 + 4 * int(rp2[-1]))
    with pytest.raises(trw.TrwError, match="2\\^31"):
        trw.DiskGraph(path2, 0)


def _write_raw(path, magic=b"TRWCSR1\0", n=3, m=2, flags=0, rp=(0, 1, 2, 2), col=(1, 2), pad=0):
    with open(path, "wb") as f:
        f.write(magic)
        f.write(np.array([n, m, flags], np.uint64).tobytes())
        f.write(np.array(rp, np.int64).tobytes())
        f.write(np.array(col, np.int32).tobytes())
        f.write(b"\0" * pad)


@pytest.mark.parametrize("case", ["magic", "short", "long", "rp0", "rpn", "decreasing", "n0", "flags"])
def test_malformed_files_are_refused(tmp_path, case):
    path = str(tmp_path / "bad.csr")
    kw = {"magic": dict(magic=b"TRWCSR2\0"), "short": dict(col=(1,)), "long": dict(pad=4),
          "rp0": dict(rp=(1, 1, 2, 2)), "rpn": dict(rp=(0, 1, 1, 1)), "decreasing": dict(rp=(0, 2, 1, 2)),
          "n0": dict(n=0, rp=(0,), m=0, col=()), "flags": dict(flags=4)}[case]
    _write_raw(path, **kw)
    with pytest.raises(trw.TrwError) as ei:
        trw.DiskGraph(path, 0)
    assert ei.value.status == _abi.TRW_E_INVALID


def test_open_argument_errors(tmp_path):
    with pytest.raises(trw.TrwError):
        trw.DiskGraph(str(tmp_path / "missing.csr"), 0)
    path = str(tmp_path / "ok.csr")
    _write_raw(path)
    with pytest.raises(trw.TrwError, match="part_edges"):
        trw.DiskGraph(path, 1 << 31)
    with pytest.raises(trw.TrwError):
        trw.write_disk_graph(str(tmp_path / "x.csr"), np.zeros(1, np.int64), np.zeros(0, np.int32))   # n = 0


def test_walk_argument_checks(tmp_path):
    g = small_graph()
    path_w = str(tmp_path / "w.csr")
    path_plain = str(tmp_path / "p.csr")
    trw.write_disk_graph(path_w, g.row_ptr, g.col, g.weight, g.label)
    trw.write_disk_graph(path_plain, g.row_ptr, g.col)
    Gw, Gp = trw.DiskGraph(path_w, 500), trw.DiskGraph(path_plain, 500)
    # Node2Vec waits under pairs of partitions: at most 1024 partitions, at least 2 resident
    n2v = trw.make_params("node2vec", "orej", 10, 1, n2v_thr_q16=(16384, 32768, 65536))
    assert Gw.walk_bytes(n2v, 10, 1) == Gw.walk_bytes(n2v, 10, 2)
    with pytest.raises(trw.TrwError, match="thresholds"):
        Gw.walk_bytes(trw.make_params("node2vec", "orej", 10, 1, n2v_thr_q16=(0, 1, 1)), 10)
    with pytest.raises(trw.TrwError, match="O-REJ"):
        Gw.walk_bytes(trw.make_params("node2vec", "alias", 10, 1), 10)
    big = synth.rmat(12, 8, False, 79)
    path_big = str(tmp_path / "big.csr")
    trw.write_disk_graph(path_big, big.row_ptr, big.col)
    many = trw.DiskGraph(path_big, 1)                   # about one partition per row: more than 1024
    assert many.parts > 1024
    with pytest.raises(trw.TrwError) as ei:
        many.walk_bytes(n2v, 10)
    assert ei.value.status == _abi.TRW_E_UNSUPPORTED
    many.walk_bytes(trw.make_params("deepwalk", "naive", 10, 1), 10)   # other walks take any count
    many.close()
    for sampler in ("alias", "its", "rej"):
        with pytest.raises(trw.TrwError, match="weights"):
            Gp.walk_bytes(trw.make_params("deepwalk", sampler, 10, 1), 10)
        Gw.walk_bytes(trw.make_params("deepwalk", sampler, 10, 1), 10)
    with pytest.raises(trw.TrwError, match="labels"):
        Gp.walk_bytes(trw.make_params("metapath", "its", 10, 1, schema=(0, 1)), 10)
    d, h = Gw.walk_bytes(trw.make_params("metapath", "its", 10, 1, schema=(0, 1)), 10)
    assert d > 0 and h > 0
    # the pinned buffer holds the largest partition: its row offsets, destinations and labels
    biggest = max(Gw.partition(i)[3] - Gw.partition(i)[2] for i in range(Gw.parts))
    assert h >= 5 * biggest
    # device bytes grow by one slot's worth per resident partition, up to the partition count
    one = Gw.walk_bytes(trw.make_params("deepwalk", "alias", 10, 1), 10, 1)[0]
    two = Gw.walk_bytes(trw.make_params("deepwalk", "alias", 10, 1), 10, 2)[0]
    slot = two - one
    assert slot >= 4 * (g.n + 1) + (4 + 4 + 32) * biggest
    assert Gw.walk_bytes(trw.make_params("deepwalk", "alias", 10, 1), 10, Gw.parts)[0] == one + (Gw.parts - 1) * slot
    assert Gw.walk_bytes(trw.make_params("deepwalk", "alias", 10, 1), 10, 10 ** 6)[0] == one + (Gw.parts - 1) * slot
    assert Gw.walk_bytes(trw.make_params("deepwalk", "alias", 10, 1), 10, 0)[0] == one
    # nq = 0 returns at once (no device work), with zero stats
    stats = _abi.trw_disk_walk_stats()
    p = trw.make_params("deepwalk", "naive", 10, 1)
    assert _abi.trw_disk_walk(Gp.handle, ctypes.byref(p), None, 0, 0, None, 11, None, None, 1, None, 0, None, 0,
                              ctypes.byref(stats), None) == 0
    assert stats.as_dict() == {"runs": 0, "loads": 0, "bytes_read": 0, "read_ns": 0, "total_ns": 0}
    # path_stride below max_len + 1
    assert _abi.trw_disk_walk(Gp.handle, ctypes.byref(p), None, 0, 0, None, 10, None, None, 1, None, 0, None, 0,
                              None, None) == _abi.TRW_E_INVALID
    Gw.close()
    Gp.close()


def test_use_after_close_is_an_error(tmp_path):
    """A closed DiskGraph passes a NULL handle: every call reports TRW_E_INVALID, and a
    second close does nothing."""
    path = str(tmp_path / "c.csr")
    _write_raw(path)
    G = trw.DiskGraph(path, 0)
    G.close()
    G.close()
    for call in (lambda: G.partition(0), lambda: G.walk_bytes(trw.make_params("deepwalk", "naive", 4, 1), 8)):
        with pytest.raises(trw.TrwError, match="NULL") as ei:
            call()
        assert ei.value.status == _abi.TRW_E_INVALID
