"""The C ABI driven from a plain C program (tests/c_abi/walk_from_c.c: hipMalloc,
graph, ALIAS table, PPR walk, end counts, top-k, the walk streamed to a file,
a server with device and host requests, the walk from the graph written to a
CSR file; no Python in the process), its outputs compared with the oracle."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import paper_2107_11983_amd as trw
import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BIN = os.path.join(HERE, "c_abi", "walk_from_c")


def test_c_program_matches_oracle(tmp_path):
    assert os.path.exists(BIN), "tests/c_abi/walk_from_c is built by __graft_entry__.build()"
    g = synth.rmat(11, 16, False, 0xC0DE)
    synth.attach_attrs(g, 0xC0DE ^ 5, weights=True)
    src = np.concatenate([synth.sources(20000, g.n, 3), np.array([-1, g.n], np.int32)]).astype(np.int32)
    max_len, seed, stop = 64, 0xABCDEF, oracle.stop_q32(0.2)
    (tmp_path / "meta.txt").write_text(f"{g.n} {g.m} {len(src)} {max_len} {seed} {stop}\n")
    for name, arr in (("row_ptr", g.row_ptr.astype(np.int32)), ("col", g.col.astype(np.int32)),
                      ("weight", g.weight.astype(np.uint32)), ("sources", src)):
        arr.tofile(tmp_path / name)
    print(f"  running {BIN} on n={g.n} m={g.m} nq={len(src)}", flush=True)
    r = subprocess.run([BIN, str(tmp_path)], capture_output=True, text=True, timeout=120)
    sys.stdout.write(r.stdout)
    assert r.returncode == 0, r.stderr
    printed = r.stdout
    nq, stride = len(src), max_len + 1
    L = np.fromfile(tmp_path / "lengths", np.uint32)
    S = np.fromfile(tmp_path / "status", np.uint8)
    P = np.fromfile(tmp_path / "paths", np.int32).reshape(nq, stride)
    thr, al = oracle.alias_build(g.row_ptr, g.weight)
    ref = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.PPR, oracle.ALIAS, max_len, seed, stop_q32=stop),
                      src, thr=thr, alias=al)
    assert np.array_equal(L, ref.lengths) and np.array_equal(S, ref.status)
    ok = ref.status != oracle.ST_BAD_SOURCE
    mask = (np.arange(stride)[None, :] <= ref.lengths[:, None]) & ok[:, None]
    assert np.array_equal(P[mask], ref.paths[mask])
    counts, skipped = oracle.end_counts(g.n, ref.paths, ref.lengths, ref.status)
    assert skipped == 2
    assert np.array_equal(np.fromfile(tmp_path / "counts", np.uint32), counts[0])
    ids, vals = oracle.topk(counts[0], 10)
    assert np.array_equal(np.fromfile(tmp_path / "top_ids", np.int32), ids)
    assert np.array_equal(np.fromfile(tmp_path / "top_vals", np.uint32), vals)

    # the same walk, streamed to disk by trw_chunk_to_fd in chunks of 4097 queries
    chunks = list(trw.read_stream_file(str(tmp_path / "stream.bin")))
    assert [c["nq"] for c in chunks] == [min(4097, nq - i) for i in range(0, nq, 4097)]
    lo = 0
    for c in chunks:
        n, off, ent = c["nq"], c["offsets"], c["entries"]
        assert c["qid_base"] == lo
        assert np.array_equal(c["lengths"], ref.lengths[lo:lo + n]) and np.array_equal(c["status"], ref.status[lo:lo + n])
        for i in range(n):
            q = lo + i
            want = ref.paths[q, :ref.lengths[q] + 1] if ref.status[q] != oracle.ST_BAD_SOURCE else ref.paths[q, :0]
            assert np.array_equal(ent[off[i]:off[i + 1]], want), q
        lo += n
    assert lo == nq

    # six served requests: PPR ALIAS, DeepWalk ALIAS, Node2Vec O-REJ in turn, seed + i,
    # sources [i nq / 6, (i + 1) nq / 6) with qid_base their first index
    thr_n2v = (16384, 32768, 65536)
    assert tuple(oracle.n2v_thresholds(2.0, 0.5)) == thr_n2v
    for i in range(6):
        a, b = nq * i // 6, nq * (i + 1) // 6
        kind = i % 3
        ml = max_len if kind == 0 else 40
        op = (oracle.WalkParams(oracle.PPR, oracle.ALIAS, ml, seed + i, stop_q32=stop) if kind == 0 else
              oracle.WalkParams(oracle.DEEPWALK, oracle.ALIAS, ml, seed + i) if kind == 1 else
              oracle.WalkParams(oracle.NODE2VEC, oracle.OREJ, ml, seed + i, n2v_thr_q16=thr_n2v))
        kw = dict(thr=thr, alias=al) if kind < 2 else {}
        r = oracle.walk(g.row_ptr, g.col, op, src[a:b], qid_base=a, **kw)
        Ls = np.fromfile(tmp_path / f"srv{i}_lengths", np.uint32)
        Ss = np.fromfile(tmp_path / f"srv{i}_status", np.uint8)
        Ps = np.fromfile(tmp_path / f"srv{i}_paths", np.int32).reshape(b - a, ml + 1)
        assert np.array_equal(Ls, r.lengths) and np.array_equal(Ss, r.status), i
        ok = r.status != oracle.ST_BAD_SOURCE
        m = (np.arange(ml + 1)[None, :] <= r.lengths[:, None]) & ok[:, None]
        assert np.array_equal(Ps[m], r.paths[m]), i
    assert (np.fromfile(tmp_path / "srv5_status", np.uint8)[-2:] == oracle.ST_BAD_SOURCE).all()

    # the same PPR walk from the graph written to a CSR file, 2 partitions resident
    Ld = np.fromfile(tmp_path / "disk_lengths", np.uint32)
    Sd = np.fromfile(tmp_path / "disk_status", np.uint8)
    Pd = np.fromfile(tmp_path / "disk_paths", np.int32).reshape(nq, stride)
    assert np.array_equal(Ld, ref.lengths) and np.array_equal(Sd, ref.status)
    assert np.array_equal(Pd[mask], ref.paths[mask])
    parts = trw.DiskGraph(str(tmp_path / "graph.csr"), g.m // 5).parts
    assert parts >= 5 and f"disk walk: {parts} partitions" in printed
