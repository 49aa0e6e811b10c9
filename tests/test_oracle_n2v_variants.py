"""Pins of the oracle's two further Node2Vec samplers (test infrastructure on the CPU).

* Weighted Node2Vec by rejection (Random Walk based Algorithms, Node2Vec: the
  transition weight is the edge weight times the second-order factor;
  Sampling Methods, rejection sampling with the row's largest weight as the
  per-vertex bound).
* Node2Vec by ITS over weights computed at each step (Analysis: ITS is the
  sampler the paper recommends for dynamic walks).

Each is checked against what the paper and the mathematics fix: the exact
transition law (chi-squared per state, and every path of three moves by
enumeration), the expected number of darts, and identities with walks the
other pins already hold: unit weights give unweighted Node2Vec bit for bit,
p = q = 1 gives the first-order walks (REJ; NAIVE on rows below 2^16 slots,
ITS on unit weights above), and scaling every weight leaves the paths alone.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from helpers import edge_index, star, undirected, zoo

P_MIN = 1e-6
N_STAT = 200_000


def _walk(g, sampler, max_len, sources, seed=1, thr=(65536, 65536, 65536), weight=None, qid_base=0):
    params = oracle.WalkParams(algo=oracle.NODE2VEC, sampler=sampler, max_len=max_len, seed=seed,
                               n2v_thr_q16=tuple(thr))
    kw = {}
    if sampler == oracle.REJ:
        w = g.weight if weight is None else weight
        kw = dict(weight=w, pmax=oracle.rej_build(g.row_ptr, w))
    return oracle.walk(g.row_ptr, g.col, params, np.asarray(sources, np.int32), qid_base=qid_base, **kw)


def _chi2(counts, probs):
    counts = np.asarray(counts, np.float64)
    probs = np.asarray(probs, np.float64)
    keep = probs > 0
    assert counts[~keep].sum() == 0, "mass on a zero-probability outcome"
    if keep.sum() == 1:
        return 1.0
    exp = probs[keep] / probs[keep].sum() * counts.sum()
    return stats.chisquare(counts[keep], exp).pvalue


def _alpha(g, prev, x, p, q):
    """The second-order factor of the transition equation (reals)."""
    if x == prev:
        return 1.0 / p
    if edge_index(g, prev, x) >= 0:
        return 1.0
    return 1.0 / q


def _nbrs(g, v):
    return [int(x) for x in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]]


def _w(g, u, x):
    return float(g.weight[edge_index(g, u, x)])


@pytest.fixture(scope="module")
def rmat(synth_lib):
    g = synth.rmat(10, 12, True, 0xA11CE)
    synth.attach_attrs(g, 0xA11CE ^ 1, weights=True)
    return g


# --------------------------------------------------------------------------- identities
def test_weighted_unit_weights_is_unweighted_orej(rmat):
    """w = 1 everywhere: p* = 1 and the hit test r1 < a * 2^16 is O-REJ's (r1 >> 16) < a."""
    g = rmat
    src = np.arange(g.n, dtype=np.int32)
    thr = oracle.n2v_thresholds(2.0, 0.5)
    a = _walk(g, oracle.REJ, 40, src, thr=thr, weight=np.ones(g.m, np.uint32))
    b = _walk(g, oracle.OREJ, 40, src, thr=thr)
    assert np.array_equal(a.paths, b.paths) and np.array_equal(a.lengths, b.lengths)
    assert np.array_equal(a.status, b.status)
    assert a.counters["orej_trials"] == b.counters["orej_trials"]


def test_weighted_p_q_one_is_rej(rmat):
    """p = q = 1: every factor is 65536, so a dart hits iff r1 * p* < w * 2^32, REJ's test."""
    g = rmat
    src = np.arange(g.n, dtype=np.int32)
    a = _walk(g, oracle.REJ, 40, src, thr=oracle.n2v_thresholds(1.0, 1.0))
    pr = oracle.WalkParams(oracle.DEEPWALK, oracle.REJ, 40, 1)
    b = oracle.walk(g.row_ptr, g.col, pr, src, weight=g.weight, pmax=oracle.rej_build(g.row_ptr, g.weight))
    assert np.array_equal(a.paths, b.paths) and np.array_equal(a.lengths, b.lengths)
    assert a.counters["orej_trials"] == b.counters["rej_trials"]


def test_weighted_scaling_leaves_paths(rmat):
    g = rmat
    src = np.arange(g.n, dtype=np.int32)
    thr = oracle.n2v_thresholds(0.5, 2.0)
    a = _walk(g, oracle.REJ, 30, src, thr=thr)
    b = _walk(g, oracle.REJ, 30, src, thr=thr, weight=g.weight * np.uint32(1000003))
    assert np.array_equal(a.paths, b.paths)


def test_its_p_q_one_is_naive(rmat):
    """p = q = 1 on rows below 2^16 slots: W = 65536 d < 2^32, the draw floor(r0 W / 2^32)
    lands in slot floor(r0 d / 2^32), NAIVE's."""
    g = rmat
    assert g.degrees().max() < 65536
    src = np.arange(g.n, dtype=np.int32)
    a = _walk(g, oracle.ITS, 40, src, thr=oracle.n2v_thresholds(1.0, 1.0))
    b = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.DEEPWALK, oracle.NAIVE, 40, 1), src)
    assert np.array_equal(a.paths, b.paths) and np.array_equal(a.lengths, b.lengths)


@pytest.mark.parametrize("f", [1, 3])
def test_its_equal_small_factors_is_naive(rmat, f):
    """Every later move weighs f per slot (thresholds (f, f, f)): W = f d, the draw
    t = floor(r0 f d / 2^32) and the slot floor(t / f) = floor(r0 d / 2^32), NAIVE's.  With
    f = 1 the draw is the slot itself, so a running-sum boundary is met on every move."""
    g = rmat
    src = np.arange(g.n, dtype=np.int32)
    a = _walk(g, oracle.ITS, 30, src, thr=(f, f, f))
    b = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.DEEPWALK, oracle.NAIVE, 30, 1), src)
    assert np.array_equal(a.paths, b.paths) and np.array_equal(a.lengths, b.lengths)


def test_its_p_q_one_large_row_is_unit_weight_its(oracle_lib):
    """A hub of 70,000 slots: W = 65536 d >= 2^32 takes the 64-bit draw, whose slot is
    floor(r d / 2^64), the ITS walk's on unit weights; leaves (d = 1) agree trivially."""
    d = 70_000
    g = star(d)
    src = np.zeros(3000, np.int32)
    a = _walk(g, oracle.ITS, 6, src, thr=oracle.n2v_thresholds(1.0, 1.0))
    ones = np.ones(g.m, np.uint32)
    pr = oracle.WalkParams(oracle.DEEPWALK, oracle.ITS, 6, 1)
    b = oracle.walk(g.row_ptr, g.col, pr, src, prefix=oracle.its_build(g.row_ptr, ones))
    assert np.array_equal(a.paths, b.paths)
    assert len(np.unique(a.paths[:, 1])) > 2500        # the hub's moves spread over its leaves


# --------------------------------------------------------------------------- laws
@pytest.mark.parametrize("pq", [(2.0, 0.5), (0.5, 2.0), (4.0, 1.0)])
@pytest.mark.parametrize("sampler", ["weighted", "its"])
def test_second_order_law(oracle_lib, pq, sampler):
    """From a fixed first move, the second move follows w_x * a(prev, x) (weighted) or
    a(prev, x) (ITS, unweighted), normalised over the row."""
    p, q = pq
    g = zoo()["tri_tail"]
    thr = oracle.n2v_thresholds(p, q)
    s = 2
    smp = oracle.REJ if sampler == "weighted" else oracle.ITS
    r = _walk(g, smp, 2, np.full(N_STAT, s), seed=42, thr=thr)
    for v in np.unique(r.paths[:, 1]):
        sel = r.paths[:, 1] == v
        probs = np.zeros(g.n)
        for x in _nbrs(g, v):
            probs[x] = _alpha(g, s, x, p, q) * (_w(g, v, x) if sampler == "weighted" else 1.0)
        counts = np.bincount(r.paths[sel, 2], minlength=g.n)
        assert _chi2(counts, probs) > P_MIN, (pq, sampler, v)


@pytest.mark.parametrize("sampler", ["weighted", "its"])
def test_full_path_law_brute_force(oracle_lib, sampler):
    """Every path of 3 moves from each source, its probability by enumeration: the first
    move follows w (weighted) or is uniform (ITS), the later ones the second-order law."""
    p, q = 2.0, 0.5
    g = zoo()["tri_tail"]
    thr = oracle.n2v_thresholds(p, q)
    wt = (lambda u, x: _w(g, u, x)) if sampler == "weighted" else (lambda u, x: 1.0)
    smp = oracle.REJ if sampler == "weighted" else oracle.ITS
    for s in (0, 3):
        law = {}
        w0 = {a: wt(s, a) for a in _nbrs(g, s)}
        for a in _nbrs(g, s):
            wb = {x: wt(a, x) * _alpha(g, s, x, p, q) for x in _nbrs(g, a)}
            for b in _nbrs(g, a):
                wc = {x: wt(b, x) * _alpha(g, a, x, p, q) for x in _nbrs(g, b)}
                for c in _nbrs(g, b):
                    law[(a, b, c)] = (w0[a] / sum(w0.values())) * wb[b] / sum(wb.values()) * wc[c] / sum(wc.values())
        r = _walk(g, smp, 3, np.full(N_STAT, s), seed=70 + s, thr=thr)
        keys = list(law)
        idx = {k: i for i, k in enumerate(keys)}
        counts = np.zeros(len(keys))
        for row in r.paths[:, 1:4]:
            counts[idx[tuple(int(x) for x in row)]] += 1
        assert abs(sum(law.values()) - 1) < 1e-12
        assert _chi2(counts, [law[k] for k in keys]) > P_MIN, (sampler, s)


@pytest.mark.parametrize("weights", [(1, 1, 2, 3, 5, 200), (4, 4, 4, 3), (1, 255)])
def test_weighted_expected_darts_first_move(oracle_lib, weights):
    """First move (factor 65536 everywhere): darts per move = d * p* / sum w (rejection)."""
    g = star(len(weights), weights=weights)
    N = 100_000
    r = _walk(g, oracle.REJ, 1, np.zeros(N, np.int32), seed=31)
    d, pstar, W = len(weights), max(weights), sum(weights)
    E = d * pstar / W
    mean = r.counters["orej_trials"] / N
    se = math.sqrt(max((1 - 1 / E) * E * E, 1e-12) / N)
    assert abs(mean - E) < 5 * se + 1e-12, (mean, E)
    assert _chi2(np.bincount(r.paths[:, 1], minlength=g.n), [0] + list(weights)) > P_MIN


def test_weighted_expected_darts_second_move(oracle_lib):
    """Second move from a fixed state: darts = d * p* * 65536 / sum(w_x * a_x)."""
    p, q = 2.0, 0.5
    # 0 -> 1 is 0's only edge; 1's neighbours 0, 2, 3, 4, 5 with weights 7, 1, 30, 2, 9;
    # 2 and 3 are adjacent to 0 (so their factor is 1), 4 and 5 are not (1/q)
    pairs = [(0, 1), (1, 2), (1, 3), (1, 4), (1, 5), (0, 2), (0, 3)]
    g = undirected(6, pairs, weights=[7, 1, 30, 2, 9, 5, 5])
    # force the first move: only 0 -> 1 is taken when 0's other edges weigh 0
    w = g.weight.copy()
    w[edge_index(g, 0, 2)] = 0
    w[edge_index(g, 0, 3)] = 0
    thr = oracle.n2v_thresholds(p, q)
    N = 100_000
    r = _walk(g, oracle.REJ, 2, np.zeros(N, np.int32), seed=5, thr=thr, weight=w)
    assert (r.paths[:, 1] == 1).all()
    first = 3 * 7 / 7                          # first move: d = 3, p* = 7, sum w = 7
    xs = _nbrs(g, 1)
    wa = [w[edge_index(g, 1, x)] * thr[0 if x == 0 else (1 if edge_index(g, 0, x) >= 0 else 2)] for x in xs]
    E = len(xs) * max(w[g.row_ptr[1]:g.row_ptr[2]]) * 65536 / sum(wa)
    mean2 = r.counters["orej_trials"] / N - first
    se = math.sqrt((1 - 1 / E) * E * E / N)
    assert abs(mean2 - E) < 5 * se, (mean2, E)


def test_weighted_zero_weights(oracle_lib):
    """A zero-weight edge is never taken; a row whose weights are all zero is a dead end."""
    edges = [(0, 1), (0, 2), (0, 3), (1, 0), (2, 0), (2, 4), (3, 0)]
    g = synth.from_edges(5, edges, [0, 5, 0, 1, 0, 0, 1])
    r = _walk(g, oracle.REJ, 4, np.zeros(2000, np.int32), seed=8, thr=oracle.n2v_thresholds(2.0, 0.5))
    assert (r.paths[:, 1] == 2).all()
    assert (r.lengths == 1).all() and (r.status == oracle.ST_DEAD_END).all()


def test_its_reads_whole_rows(oracle_lib):
    """Dynamic ITS weighs every slot of the row at each move (the paper's O(d) per step for
    dynamic walks): one adjacency test per slot and move, plus the cumulative pass."""
    g = zoo()["k4"]
    N = 1000
    r = _walk(g, oracle.ITS, 3, np.zeros(N, np.int32), thr=oracle.n2v_thresholds(2.0, 0.5))
    assert r.counters["moves"] == 3 * N
    assert 1 <= r.counters["its_probes"] / r.counters["moves"] <= 3      # slots scanned up to the pick
