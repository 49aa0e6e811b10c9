"""Pins for the oracle's PPR estimate and top-k (Random Walk based Algorithms, PPR:
a vertex's score for a source is the share of the source's queries that end there).

  * end counts on hand-built path arrays with the expected counts written out,
    including groups, bad sources and out-of-range ends;
  * the directed cycle, where a walk of L moves from s ends at (s + L) mod n;
  * the end-count distribution against power iteration on a small weighted graph;
  * top-k on a hand-worked example and, on random inputs with many ties,
    against the defining property checked by loops (every vertex left out
    ranks below every vertex taken).
"""
import numpy as np
import pytest

import oracle
import synth

N_STAT = 200_000


def test_end_counts_hand_built(oracle_lib):
    n = 6
    paths = np.full((5, 4), -1, np.int32)
    paths[0, :3] = [0, 2, 5]          # 2 moves, ends at 5
    paths[1, :1] = [3]                # dead end at the source: ends at 3
    paths[2, :4] = [1, 2, 3, 4]       # 3 moves, ends at 4
    paths[3, :1] = [9]                # bad source: skipped
    paths[4, :2] = [5, 5]             # ends at 5
    lengths = np.array([2, 0, 3, 0, 1], np.uint32)
    status = np.array([2, 3, 1, 4, 2], np.uint8)
    c, skipped = oracle.end_counts(n, paths, lengths, status)
    assert skipped == 1
    assert c.tolist() == [[0, 0, 0, 1, 1, 2]]
    c, skipped = oracle.end_counts(n, paths, lengths, status, group=2)
    assert skipped == 1
    assert c.tolist() == [[0, 0, 0, 1, 0, 1],     # queries 0, 1
                          [0, 0, 0, 0, 1, 0],     # queries 2, 3
                          [0, 0, 0, 0, 0, 1]]     # query 4
    # counts accumulate over calls
    c2, _ = oracle.end_counts(n, paths, lengths, status, group=2, counts=c)
    assert c2 is c and c.sum() == 8
    # an end outside [0, n), or a length past the row, is skipped
    bad = paths.copy()
    bad[0, 2] = 77
    c, skipped = oracle.end_counts(n, bad, np.array([2, 0, 3, 0, 9], np.uint32), status)
    assert skipped == 3 and c.tolist() == [[0, 0, 0, 1, 1, 0]]


def test_end_counts_directed_cycle(oracle_lib):
    n = 7
    g = synth.from_edges(n, [(i, (i + 1) % n) for i in range(n)], [1] * n)
    src = np.array([0, 3, 6, 2] * 500, np.int32)
    p = oracle.WalkParams(oracle.PPR, oracle.NAIVE, 40, 5, stop_q32=oracle.stop_q32(0.3))
    r = oracle.walk(g.row_ptr, g.col, p, src)
    c, skipped = oracle.end_counts(n, r.paths, r.lengths, r.status)
    assert skipped == 0
    expect = np.bincount((src.astype(np.int64) + r.lengths) % n, minlength=n)
    assert np.array_equal(c[0], expect)


def test_end_counts_ppr_power_iteration(oracle_lib):
    """Scores = counts / N against the exact end law (the PPR walk, power iteration)."""
    edges = [(0, 1), (0, 2), (1, 2), (1, 3), (2, 0), (2, 4), (3, 0), (3, 5), (4, 1), (4, 3)]
    w = [5, 1, 2, 2, 1, 7, 3, 1, 4, 4]
    g = synth.from_edges(6, edges, w)
    alpha, L, s = 0.2, 256, 1
    thr, al = oracle.alias_build(g.row_ptr, g.weight)
    p = oracle.WalkParams(oracle.PPR, oracle.ALIAS, L, 77, stop_q32=oracle.stop_q32(alpha))
    r = oracle.walk(g.row_ptr, g.col, p, np.full(N_STAT, s, np.int32), thr=thr, alias=al)
    c, _ = oracle.end_counts(g.n, r.paths, r.lengths, r.status)
    # exact law: sum over k of alpha (1 - alpha)^(k-1) e_s P^k, plus the capped tail; 5 dangles
    P = np.zeros((6, 6))
    for (u, v), x in zip(edges, w):
        P[u, v] = x
    P[5, 5] = 1.0
    P /= P.sum(axis=1, keepdims=True)
    x = np.zeros(6)
    x[s] = 1.0
    pi = np.zeros(6)
    for k in range(1, L + 1):
        x = x @ P
        pi += alpha * (1 - alpha) ** (k - 1) * x
    pi += (1 - alpha) ** L * x
    emp = c[0] / N_STAT
    tol = 5 * np.sqrt(pi * (1 - pi) / N_STAT) + 1e-9
    assert (np.abs(emp - pi) <= tol).all(), (emp, pi)


def test_topk_hand_worked(oracle_lib):
    counts = np.array([3, 7, 7, 0, 5, 7, 1], np.uint32)
    ids, vals = oracle.topk(counts, 4)
    assert ids.tolist() == [1, 2, 5, 4] and vals.tolist() == [7, 7, 7, 5]
    ids, vals = oracle.topk(counts, 7)
    assert ids.tolist() == [1, 2, 5, 4, 0, 6, 3]
    ids, vals = oracle.topk(counts, 0)
    assert len(ids) == 0
    with pytest.raises(ValueError):
        oracle.topk(counts, 8)


def _ranks_before(a, b):
    """(count, id) a ranks before b: larger count, or equal count and smaller id."""
    return a[0] > b[0] or (a[0] == b[0] and a[1] < b[1])


@pytest.mark.parametrize("seed", range(6))
def test_topk_defining_property(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    counts = rng.integers(0, 6, size=n).astype(np.uint32)      # many ties
    if seed == 5:
        counts[:] = 4                                          # all tied
    for k in sorted({0, 1, n // 3, n - 1, n} - {-1}):
        ids, vals = oracle.topk(counts, k)
        assert len(set(ids.tolist())) == k
        for i in range(k):
            assert vals[i] == counts[ids[i]]
            if i:
                assert _ranks_before((vals[i - 1], ids[i - 1]), (vals[i], ids[i]))
        taken = set(ids.tolist())
        if k:
            last = (int(vals[-1]), int(ids[-1]))
            for v in range(n):
                if v not in taken:
                    assert _ranks_before(last, (int(counts[v]), v))
