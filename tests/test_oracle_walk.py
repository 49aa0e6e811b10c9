"""Pins for the oracle's walker.

Each check is tied to something outside the oracle's own code:
  * hand-worked first moves from the Philox known-answer block (golden file);
  * invariants of the execution paradigm (every hop is an edge, termination rules);
  * exact special cases that reduce one algorithm to another;
  * chi-squared tests of empirical transition frequencies against exact
    probabilities (NAIVE, ALIAS, ITS, Node2Vec's second-order rule, MetaPath);
  * the full path law on small graphs by brute-force enumeration;
  * PPR end-vertex distribution against power iteration, and the expected
    walk length of 5 at stop probability 0.2 that the paper states (Evaluation
    of Step Interleaving);
  * the O-REJ and REJ expected number of darts d * p* / sum p (Sampling
    Methods).
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from helpers import edge_index, golden_path, star, transition_matrix, undirected, zoo

P_MIN = 1e-6   # chi-squared rejection level; seeds are fixed, so this is deterministic


def _walk(g, algo, sampler, max_len, sources, seed=1, qid_base=0, qids=None, stop=0,
          thr_q16=(65536, 65536, 65536), schema=(), tables=None):
    params = oracle.WalkParams(algo=algo, sampler=sampler, max_len=max_len, seed=seed,
                               stop_q32=stop, n2v_thr_q16=thr_q16, schema=tuple(schema))
    kw = {}
    if sampler == oracle.ALIAS:
        t, a = tables if tables is not None else oracle.alias_build(g.row_ptr, g.weight)
        kw.update(thr=t, alias=a)
    if sampler == oracle.ITS and algo != oracle.METAPATH:
        kw.update(prefix=tables if tables is not None else oracle.its_build(g.row_ptr, g.weight))
    if sampler == oracle.REJ:
        kw.update(weight=g.weight, pmax=tables if tables is not None else oracle.rej_build(g.row_ptr, g.weight))
    if algo == oracle.METAPATH:
        kw.update(label=g.label)
    return oracle.walk(g.row_ptr, g.col, params, np.asarray(sources, np.int32), qid_base=qid_base,
                       qids=qids, **kw)


def _chi2(counts, probs):
    counts = np.asarray(counts, np.float64)
    probs = np.asarray(probs, np.float64)
    keep = probs > 0
    assert counts[~keep].sum() == 0, "mass on a zero-probability outcome"
    if keep.sum() == 1:          # a single possible outcome: all mass must be there
        return 1.0
    exp = probs[keep] / probs[keep].sum() * counts.sum()
    return stats.chisquare(counts[keep], exp).pvalue


# --------------------------------------------------------------------------- golden
def _golden_walk_lines():
    for line in open(golden_path("walk_worked_examples.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            kind, *kv = line.split()
            yield kind, dict(x.split("=") for x in kv)


def test_worked_first_moves(oracle_lib):
    n = 0
    for kind, kv in _golden_walk_lines():
        if kind == "naive":
            d, j = int(kv["d"]), int(kv["j"])
            g = star(d)
            r = _walk(g, oracle.DEEPWALK, oracle.NAIVE, 1, [0], seed=0)
            assert r.paths[0, 1] == j + 1
        elif kind in ("its", "alias"):
            w = [int(x) for x in kv["weights"].split(",")]
            g = star(len(w), weights=w)
            s = oracle.ITS if kind == "its" else oracle.ALIAS
            r = _walk(g, oracle.DEEPWALK, s, 1, [0], seed=0)
            assert r.paths[0, 1] == int(kv["i"]) + 1, (kind, kv)
        elif kind == "rej":
            w = [int(x) for x in kv["weights"].split(",")]
            g = star(len(w), weights=w)
            r = _walk(g, oracle.DEEPWALK, oracle.REJ, 1, [0], seed=0)
            assert (r.counters["rej_trials"] == 1) == bool(int(kv["hit"])), kv
            if "i" in kv:
                assert r.paths[0, 1] == int(kv["i"]) + 1, kv
        elif kind == "ppr":
            g = star(10)
            r = _walk(g, oracle.PPR, oracle.NAIVE, 5, [0], seed=0, stop=int(kv["stop_q32"]))
            stopped_first = r.lengths[0] == 1 and r.status[0] == oracle.ST_STOPPED
            assert stopped_first == bool(int(kv["stopped"]))
        n += 1
    assert n == 12


# --------------------------------------------------------------------------- invariants
@pytest.fixture(scope="module")
def rmat_graphs(synth_lib):
    gs = synth.rmat(10, 12, True, 0xA11CE)
    synth.attach_attrs(gs, 0xA11CE ^ 1, weights=True, labels=5)
    gd = synth.rmat(10, 12, False, 0xB0B)
    synth.attach_attrs(gd, 0xB0B ^ 1, weights=True)
    return gs, gd


def _check_paths_are_edges(g, r, sources):
    deg = g.degrees()
    for i in range(len(sources)):
        L = int(r.lengths[i])
        p = r.paths[i]
        assert p[0] == sources[i]
        for k in range(L):
            assert edge_index(g, p[k], p[k + 1]) >= 0, (i, k)
        if r.status[i] == oracle.ST_DEAD_END:
            assert deg[p[L]] == 0 or g.label is not None
    return True


@pytest.mark.parametrize("sampler", [oracle.NAIVE, oracle.ALIAS, oracle.ITS, oracle.REJ])
def test_deepwalk_invariants(rmat_graphs, sampler):
    g, _ = rmat_graphs
    src = np.arange(g.n, dtype=np.int32)
    r = _walk(g, oracle.DEEPWALK, sampler, 20, src)
    _check_paths_are_edges(g, r, src)
    deg = g.degrees()
    for i in range(g.n):
        if deg[i] == 0:
            assert r.lengths[i] == 0 and r.status[i] == oracle.ST_DEAD_END
        else:   # symmetric: every vertex entered has an edge back
            assert r.lengths[i] == 20 and r.status[i] == oracle.ST_LENGTH
    assert r.counters["moves"] == int(r.lengths.sum())


@pytest.mark.parametrize("sampler", [oracle.NAIVE, oracle.ALIAS, oracle.ITS, oracle.REJ])
def test_ppr_invariants(rmat_graphs, sampler):
    _, g = rmat_graphs
    src = synth.sources(5000, g.n, 77)
    r = _walk(g, oracle.PPR, sampler, 256, src, stop=oracle.stop_q32(0.2))
    _check_paths_are_edges(g, r, src)
    deg = g.degrees()
    for i in range(len(src)):
        L = int(r.lengths[i])
        if r.status[i] == oracle.ST_STOPPED:
            assert L >= 1
        elif r.status[i] == oracle.ST_DEAD_END:
            assert deg[r.paths[i, L]] == 0
        else:
            assert r.status[i] == oracle.ST_LENGTH and L == 256


def test_node2vec_invariants(rmat_graphs):
    g, _ = rmat_graphs
    src = np.arange(g.n, dtype=np.int32)
    r = _walk(g, oracle.NODE2VEC, oracle.OREJ, 30, src, thr_q16=oracle.n2v_thresholds(2.0, 0.5))
    _check_paths_are_edges(g, r, src)
    deg = g.degrees()
    assert ((r.lengths == 30) == (deg > 0)).all()


def test_metapath_invariants(rmat_graphs):
    g, _ = rmat_graphs
    schema = (1, 3, 3, 0, 4)
    src = np.arange(g.n, dtype=np.int32)
    r = _walk(g, oracle.METAPATH, oracle.ITS, 100, src, schema=schema)
    _check_paths_are_edges(g, r, src)
    for i in range(g.n):
        L = int(r.lengths[i])
        p = r.paths[i]
        for k in range(L):
            assert g.label[edge_index(g, p[k], p[k + 1])] == schema[k % 5]
        if r.status[i] == oracle.ST_DEAD_END:
            lo, hi = g.row_ptr[p[L]], g.row_ptr[p[L] + 1]
            assert not (g.label[lo:hi] == schema[L % 5]).any()
        else:
            assert r.status[i] == oracle.ST_LENGTH and L == 100
    assert len(set(r.lengths.tolist())) > 10       # highly uneven lengths


def test_bad_sources(rmat_graphs):
    g, _ = rmat_graphs
    r = _walk(g, oracle.DEEPWALK, oracle.NAIVE, 5, [-1, g.n, 0, 2**31 - 1])
    assert list(r.status[[0, 1, 3]]) == [oracle.ST_BAD_SOURCE] * 3
    assert list(r.lengths[[0, 1, 3]]) == [0, 0, 0]


def test_directed_cycle_is_deterministic(oracle_lib):
    n = 7
    g = synth.from_edges(n, [(i, (i + 1) % n) for i in range(n)], weights=[3] * n)
    for sampler in (oracle.NAIVE, oracle.ALIAS, oracle.ITS):
        r = _walk(g, oracle.DEEPWALK, sampler, 25, [2, 5], seed=99)
        for i, s in enumerate([2, 5]):
            assert list(r.paths[i]) == [(s + k) % n for k in range(26)]


def test_queries_are_independent(rmat_graphs):
    """A query's walk depends only on (seed, qid, source): subsets reproduce the batch."""
    g, _ = rmat_graphs
    src = synth.sources(3000, g.n, 5)
    full = _walk(g, oracle.PPR, oracle.ALIAS, 64, src, qid_base=1000, stop=oracle.stop_q32(0.1))
    sel = np.array([0, 17, 2999, 1500, 3], dtype=np.int64)
    sub = _walk(g, oracle.PPR, oracle.ALIAS, 64, src[sel], qids=(1000 + sel).astype(np.uint64),
                stop=oracle.stop_q32(0.1))
    assert np.array_equal(sub.lengths, full.lengths[sel])
    for a, i in enumerate(sel):
        L = int(full.lengths[i]) + 1
        assert np.array_equal(sub.paths[a, :L], full.paths[i, :L])


# --------------------------------------------------------------------------- identities
def test_identity_node2vec_unit_params_is_naive(rmat_graphs):
    g, _ = rmat_graphs
    src = np.arange(g.n, dtype=np.int32)
    a = _walk(g, oracle.NODE2VEC, oracle.OREJ, 40, src, thr_q16=oracle.n2v_thresholds(1.0, 1.0))
    b = _walk(g, oracle.DEEPWALK, oracle.NAIVE, 40, src)
    assert np.array_equal(a.paths, b.paths) and np.array_equal(a.lengths, b.lengths)


def test_identity_alias_uniform_is_naive(rmat_graphs):
    g, _ = rmat_graphs
    gu = synth.CSRGraph(g.n, g.row_ptr, g.col, weight=np.full(g.m, 9, np.uint32))
    src = np.arange(g.n, dtype=np.int32)
    a = _walk(gu, oracle.DEEPWALK, oracle.ALIAS, 40, src)
    b = _walk(gu, oracle.DEEPWALK, oracle.NAIVE, 40, src)
    assert np.array_equal(a.paths, b.paths)


@pytest.mark.parametrize("algo", [oracle.DEEPWALK, oracle.PPR])
def test_identity_rej_uniform_is_naive(rmat_graphs, algo):
    """Equal weights: every first dart hits, so REJ takes NAIVE's edge and stop coin."""
    _, g = rmat_graphs
    gu = synth.CSRGraph(g.n, g.row_ptr, g.col, weight=np.full(g.m, 17, np.uint32))
    src = synth.sources(3000, g.n, 21)
    stop = oracle.stop_q32(0.2) if algo == oracle.PPR else 0
    a = _walk(gu, algo, oracle.REJ, 50, src, stop=stop)
    b = _walk(gu, algo, oracle.NAIVE, 50, src, stop=stop)
    assert np.array_equal(a.paths, b.paths) and np.array_equal(a.lengths, b.lengths)
    assert np.array_equal(a.status, b.status)
    assert a.counters["rej_trials"] == a.counters["moves"]


def test_rej_zero_weights(oracle_lib):
    """A zero-weight edge is never taken; a row whose weights are all zero is a dead end."""
    # 0 -> {1, 2, 3} with weights 0, 5, 0; 2 -> {0, 4} with weights 0, 0; 1 and 3 -> 0
    edges = [(0, 1), (0, 2), (0, 3), (1, 0), (2, 0), (2, 4), (3, 0)]
    g = synth.from_edges(5, edges, [0, 5, 0, 1, 0, 0, 1])
    r = _walk(g, oracle.DEEPWALK, oracle.REJ, 4, np.zeros(2000, np.int32), seed=8)
    assert (r.paths[:, 1] == 2).all()
    assert (r.lengths == 1).all() and (r.status == oracle.ST_DEAD_END).all()
    assert list(oracle.rej_build(g.row_ptr, g.weight)) == [5, 1, 0, 1, 0]


def test_identity_metapath_all_match_is_naive(rmat_graphs):
    g, _ = rmat_graphs
    gl = synth.CSRGraph(g.n, g.row_ptr, g.col, label=np.full(g.m, 2, np.uint8))
    src = np.arange(g.n, dtype=np.int32)
    a = _walk(gl, oracle.METAPATH, oracle.ITS, 40, src, schema=(2, 2, 2))
    b = _walk(gl, oracle.DEEPWALK, oracle.NAIVE, 40, src)
    assert np.array_equal(a.paths, b.paths) and np.array_equal(a.lengths, b.lengths)


@pytest.mark.parametrize("sampler", [oracle.NAIVE, oracle.ALIAS, oracle.ITS, oracle.REJ])
def test_identity_ppr_without_stop_is_fixed_length(rmat_graphs, sampler):
    _, g = rmat_graphs
    src = synth.sources(2000, g.n, 11)
    a = _walk(g, oracle.PPR, sampler, 33, src, stop=0)
    b = _walk(g, oracle.DEEPWALK, sampler, 33, src)
    assert np.array_equal(a.paths, b.paths) and np.array_equal(a.status, b.status)


@pytest.mark.parametrize("sampler", [oracle.ALIAS, oracle.ITS, oracle.REJ])
def test_identity_weight_scaling(rmat_graphs, sampler):
    g, _ = rmat_graphs
    g2 = synth.CSRGraph(g.n, g.row_ptr, g.col, weight=g.weight * np.uint32(1000003))
    src = np.arange(g.n, dtype=np.int32)
    a = _walk(g, oracle.DEEPWALK, sampler, 30, src)
    b = _walk(g2, oracle.DEEPWALK, sampler, 30, src)
    assert np.array_equal(a.paths, b.paths)


# --------------------------------------------------------------------------- distributions
N_STAT = 200_000


@pytest.mark.parametrize("name", ["tri_tail", "k4", "star6", "path6"])
@pytest.mark.parametrize("sampler", [oracle.NAIVE, oracle.ALIAS, oracle.ITS, oracle.REJ])
def test_first_step_law(oracle_lib, name, sampler):
    g = zoo()[name]
    P = transition_matrix(g, use_weights=sampler != oracle.NAIVE)
    for s in range(min(g.n, 3)):
        r = _walk(g, oracle.DEEPWALK, sampler, 1, np.full(N_STAT, s), seed=1234 + s)
        counts = np.bincount(r.paths[:, 1], minlength=g.n)
        assert _chi2(counts, P[s]) > P_MIN, (name, sampler, s)


def _n2v_weight(g, prev, x, p, q):
    if x == prev:
        return 1.0 / p
    if edge_index(g, prev, x) >= 0:
        return 1.0
    return 1.0 / q


@pytest.mark.parametrize("pq", [(2.0, 0.5), (0.5, 2.0), (4.0, 1.0)])
def test_node2vec_second_order_law(oracle_lib, pq):
    p, q = pq
    g = zoo()["tri_tail"]
    thr = oracle.n2v_thresholds(p, q)
    s = 2
    r = _walk(g, oracle.NODE2VEC, oracle.OREJ, 2, np.full(N_STAT, s), seed=42, thr_q16=thr)
    for v in np.unique(r.paths[:, 1]):
        sel = r.paths[:, 1] == v
        nbrs = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        probs = np.zeros(g.n)
        for x in nbrs:
            probs[x] = _n2v_weight(g, s, x, p, q)
        counts = np.bincount(r.paths[sel, 2], minlength=g.n)
        assert _chi2(counts, probs) > P_MIN, (pq, v)


def test_node2vec_full_path_law_brute_force(oracle_lib):
    """All paths of 3 moves from each source, probabilities by enumeration."""
    p, q = 2.0, 0.5
    g = zoo()["tri_tail"]
    thr = oracle.n2v_thresholds(p, q)
    for s in (0, 4):
        law = {}
        def nb(v):
            return [int(x) for x in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]]
        for a in nb(s):
            for b in nb(a):
                wb = {x: _n2v_weight(g, s, x, p, q) for x in nb(a)}
                for c in nb(b):
                    wc = {x: _n2v_weight(g, a, x, p, q) for x in nb(b)}
                    law[(a, b, c)] = (1 / len(nb(s))) * wb[b] / sum(wb.values()) * wc[c] / sum(wc.values())
        r = _walk(g, oracle.NODE2VEC, oracle.OREJ, 3, np.full(N_STAT, s), seed=7 + s, thr_q16=thr)
        keys = list(law)
        idx = {k: i for i, k in enumerate(keys)}
        counts = np.zeros(len(keys))
        for row in r.paths[:, 1:4]:
            counts[idx[tuple(int(x) for x in row)]] += 1
        assert abs(sum(law.values()) - 1) < 1e-12
        assert _chi2(counts, [law[k] for k in keys]) > P_MIN


def test_metapath_law(oracle_lib):
    g = zoo()["star6"]     # labels of 0's edges: 0 1 2 0 1 2
    for lab in (0, 1, 2):
        r = _walk(g, oracle.METAPATH, oracle.ITS, 1, np.zeros(N_STAT // 4, np.int32), seed=3,
                  schema=(lab,))
        lo, hi = g.row_ptr[0], g.row_ptr[1]
        probs = np.zeros(g.n)
        for e in range(lo, hi):
            if g.label[e] == lab:
                probs[g.col[e]] = 1.0
        counts = np.bincount(r.paths[:, 1], minlength=g.n)
        assert _chi2(counts, probs) > P_MIN
    # a label absent from the row ends the walk with no move
    r = _walk(g, oracle.METAPATH, oracle.ITS, 4, np.zeros(10, np.int32), schema=(4,))
    assert (r.lengths == 0).all() and (r.status == oracle.ST_DEAD_END).all()


def _ppr_end_law(g, s, alpha, L, use_weights):
    P = transition_matrix(g, use_weights)
    deg = g.degrees()
    for v in range(g.n):            # a walk that reaches a dangling vertex ends there
        if deg[v] == 0:
            P[v, v] = 1.0
    x = np.zeros(g.n)
    x[s] = 1.0
    end = np.zeros(g.n)
    for k in range(1, L + 1):
        x = x @ P
        end += alpha * (1 - alpha) ** (k - 1) * x
    end += (1 - alpha) ** L * x
    if deg[s] == 0:
        end = np.zeros(g.n)
        end[s] = 1.0
    return end


@pytest.mark.parametrize("sampler", [oracle.NAIVE, oracle.ALIAS, oracle.ITS, oracle.REJ])
def test_ppr_end_distribution_power_iteration(oracle_lib, sampler):
    # directed weighted graph with one dangling vertex (5)
    edges = [(0, 1), (0, 2), (1, 2), (1, 3), (2, 0), (2, 4), (3, 0), (3, 5), (4, 1), (4, 3)]
    w = [5, 1, 2, 2, 1, 7, 3, 1, 4, 4]
    g = synth.from_edges(6, edges, w)
    alpha, L = 0.2, 256
    for s in (0, 3):
        r = _walk(g, oracle.PPR, sampler, L, np.full(N_STAT, s), seed=100 + s,
                  stop=oracle.stop_q32(alpha))
        ends = r.paths[np.arange(N_STAT), r.lengths.astype(np.int64)]
        emp = np.bincount(ends, minlength=g.n) / N_STAT
        pi = _ppr_end_law(g, s, alpha, L, use_weights=sampler != oracle.NAIVE)
        tol = 5 * np.sqrt(pi * (1 - pi) / N_STAT) + 1e-9
        assert (np.abs(emp - pi) <= tol).all(), (emp, pi)


def test_ppr_expected_length_is_five(oracle_lib):
    """At stop probability 0.2 a query makes 5 moves on average (the paper's figure)."""
    g = zoo()["k4"]
    r = _walk(g, oracle.PPR, oracle.ALIAS, 256, np.zeros(N_STAT, np.int32), seed=5,
              stop=oracle.stop_q32(0.2))
    L = r.lengths.astype(np.float64)
    se = math.sqrt(0.8 / 0.2 ** 2 / N_STAT)
    assert abs(L.mean() - 5.0) < 5 * se
    counts = np.bincount(r.lengths, minlength=40)[1:40]
    probs = 0.2 * 0.8 ** np.arange(39)
    assert _chi2(counts, probs / probs.sum()) > P_MIN


@pytest.mark.parametrize("pq", [(2.0, 0.5), (0.5, 2.0)])
def test_orej_expected_trials(oracle_lib, pq):
    """Mean darts per move from a fixed state = d * p* / sum p (Sampling Methods, REJ)."""
    p, q = pq
    # 0 -> 1 is 0's only edge (forced first move); 1's neighbours: 0, 2, 3, 4, 5
    edges = [(0, 1)] + [(1, x) for x in (0, 2, 3, 4, 5)] + [(x, 1) for x in (2, 3, 4, 5)]
    g = synth.from_edges(6, edges)
    thr = oracle.n2v_thresholds(p, q)
    N = 100_000
    r = _walk(g, oracle.NODE2VEC, oracle.OREJ, 2, np.zeros(N, np.int32), seed=9, thr_q16=thr)
    weights = [_n2v_weight(g, 0, x, p, q) for x in (0, 2, 3, 4, 5)]
    pstar = max(1.0, 1 / p, 1 / q)
    E = 5 * pstar / sum(weights)
    trials_step1 = (r.counters["orej_trials"] - N) / N
    se = math.sqrt((1 - 1 / E) * E * E / N)
    assert abs(trials_step1 - E) < 5 * se, (trials_step1, E)


@pytest.mark.parametrize("weights", [(1, 1, 2, 3, 5, 200), (4, 4, 4, 3), (1, 255), (255, 1, 1, 1, 1, 1, 1, 1)])
def test_rej_expected_trials(oracle_lib, weights):
    """Mean REJ darts per move = d * p* / sum w (Sampling Methods, REJ)."""
    g = star(len(weights), weights=weights)
    N = 100_000
    r = _walk(g, oracle.DEEPWALK, oracle.REJ, 1, np.zeros(N, np.int32), seed=31)
    d, pstar, W = len(weights), max(weights), sum(weights)
    E = d * pstar / W
    mean = r.counters["rej_trials"] / N
    se = math.sqrt(max((1 - 1 / E) * E * E, 1e-12) / N)
    assert abs(mean - E) < 5 * se + 1e-12, (mean, E)
    counts = np.bincount(r.paths[:, 1], minlength=g.n)
    assert _chi2(counts, [0] + list(weights)) > P_MIN


def test_rej_table_worked_example(oracle_lib):
    """p*_v by hand for the zoo graphs: the heaviest edge of each row."""
    z = zoo()
    # tri_tail: 0:{1:3, 2:4}  1:{0:3, 2:1, 3:9}  2:{0:4, 1:1, 3:1}  3:{1:9, 2:1, 4:5}  4:{3:5}
    assert list(oracle.rej_build(z["tri_tail"].row_ptr, z["tri_tail"].weight)) == [4, 9, 4, 9, 5]
    # star6: the hub's heaviest edge is 200; each leaf has its one edge
    assert list(oracle.rej_build(z["star6"].row_ptr, z["star6"].weight)) == [200, 1, 1, 2, 3, 5, 200]


@pytest.mark.parametrize("d", [1, 2, 3, 7, 8, 1000])
def test_its_probe_bound(oracle_lib, d):
    """ITS generation is a binary search: at most ceil(log2 d) probes per move."""
    rng = np.random.default_rng(d)
    g = star(d, weights=rng.integers(1, 256, size=d))
    N = 2000
    r = _walk(g, oracle.DEEPWALK, oracle.ITS, 1, np.zeros(N, np.int32))
    assert r.counters["its_probes"] <= N * math.ceil(math.log2(d)) if d > 1 else r.counters["its_probes"] == 0
