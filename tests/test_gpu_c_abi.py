"""The C ABI driven from a plain C program (tests/c_abi/walk_from_c.c: hipMalloc,
graph, ALIAS table, PPR walk, end counts, top-k; no Python in the process),
its outputs compared with the oracle."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BIN = os.path.join(HERE, "c_abi", "walk_from_c")


def test_c_program_ppr_matches_oracle(tmp_path):
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
