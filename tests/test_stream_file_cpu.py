"""The library's file sink for streamed output (trw_chunk_to_fd) on the host:
a chunk built here is written as the documented record and read back by
read_stream_file field for field; a failing write stops the stream."""
import ctypes
import os

import numpy as np


def _chunk(abi, qid_base, lengths, status, offsets, entries):
    keep = [np.ascontiguousarray(lengths, np.uint32), np.ascontiguousarray(status, np.uint8),
            np.ascontiguousarray(offsets, np.uint64), np.ascontiguousarray(entries, np.int32)]
    c = abi.trw_chunk()
    c.qid_base = qid_base
    c.nq = len(keep[0])
    c.lengths, c.status, c.offsets, c.entries = (a.ctypes.data for a in keep)
    return c, keep


def test_chunk_records_round_trip(tmp_path):
    import paper_2107_11983_amd as trw
    abi = trw._abi
    path = str(tmp_path / "chunks.bin")
    fd = os.open(path, os.O_WRONLY | os.O_CREAT | os.O_TRUNC, 0o644)
    box = ctypes.c_int(fd)
    # chunk 1: three queries (one bad source with an empty path), nq not a multiple of 8
    c1, k1 = _chunk(abi, 1 << 40, [2, 0, 1], [1, 4, 3], [0, 3, 3, 5], [7, 8, 9, 4, 4])
    # chunk 2: eight queries, no padding after the status bytes
    L2 = np.arange(8, dtype=np.uint32)
    off2 = np.concatenate([[0], np.cumsum(L2 + 1)]).astype(np.uint64)
    c2, k2 = _chunk(abi, (1 << 40) + 3, L2, np.full(8, 1), off2, np.arange(int(off2[-1]), dtype=np.int32) - 5)
    assert abi.trw_chunk_to_fd(ctypes.byref(box), ctypes.byref(c1)) == 0
    assert abi.trw_chunk_to_fd(ctypes.byref(box), ctypes.byref(c2)) == 0
    os.close(fd)
    assert os.path.getsize(path) == (16 + 12 + 3 + 5 + 32 + 20) + (16 + 32 + 8 + 72 + 4 * int(off2[-1]))
    got = list(trw.read_stream_file(path))
    assert [c["qid_base"] for c in got] == [1 << 40, (1 << 40) + 3] and [c["nq"] for c in got] == [3, 8]
    for c, (L, S, O, E) in zip(got, (k1, k2)):
        assert np.array_equal(c["lengths"], L) and np.array_equal(c["status"], S)
        assert np.array_equal(c["offsets"], O) and np.array_equal(c["entries"], E)


def test_failing_write_stops_the_stream(tmp_path):
    import paper_2107_11983_amd as trw
    abi = trw._abi
    path = str(tmp_path / "ro.bin")
    open(path, "wb").close()
    fd = os.open(path, os.O_RDONLY)            # writes to a read-only descriptor fail
    box = ctypes.c_int(fd)
    c, _keep = _chunk(abi, 0, [1], [1], [0, 2], [3, 4])
    assert abi.trw_chunk_to_fd(ctypes.byref(box), ctypes.byref(c)) != 0
    os.close(fd)
    assert abi.trw_chunk_to_fd(None, ctypes.byref(c)) != 0
