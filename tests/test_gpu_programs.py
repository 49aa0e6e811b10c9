"""Walk programs on the GPU (C ABI trw_program_*).

DeepWalk, PPR, Node2Vec and MetaPath written as programs must give the
built-in walks' outputs bit for bit, and so the oracle's.  Weighted Node2Vec,
Node2Vec by dynamic ITS and the weighted walk by rejection, which have no
built-in walk, must give the oracle's walks of the same name bit for bit
(weights in [1, 255], with the per-vertex bound of a REJ table and with a
global bound), and follow their exact laws on small graphs.
"""
import numpy as np
import pytest
import scipy.stats
import torch

import oracle
import synth
from helpers import undirected

pytestmark = pytest.mark.gpu

trw = None


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def env():
    global trw
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2107_11983_amd as mod
    trw = mod
    torch.cuda.set_device(0)
    sym = synth.rmat(12, 16, True, 0x9A11)
    synth.attach_attrs(sym, 0x9A12, weights=True, labels=5)
    dirg = synth.rmat(12, 16, False, 0x9A13)
    synth.attach_attrs(dirg, 0x9A14, weights=True)
    out = {}
    for name, g, symmetric in (("sym", sym, True), ("dir", dirg, False)):
        G = trw.Graph(g.row_ptr, g.col, g.weight, g.label, symmetric=symmetric)
        assert G.validate() == 0
        out[name] = dict(g=g, G=G, alias=G.table("alias"), its=G.table("its"), rej=G.table("rej"),
                         eidx=G.edge_index())
    torch.cuda.synchronize()
    return out


def _np(P, L, S):
    return P.cpu().numpy(), L.cpu().numpy().view(np.uint32), S.cpu().numpy()


def _same(a, b, max_len):
    Pa, La, Sa = a
    Pb, Lb, Sb = b
    assert np.array_equal(La, Lb) and np.array_equal(Sa, Sb)
    # path rows of bad sources are left untouched (unspecified)
    mask = (np.arange(max_len + 1)[None, :] <= La[:, None]) & (Sa != 4)[:, None]
    assert np.array_equal(Pa[:, :max_len + 1][mask], Pb[:, :max_len + 1][mask])


def _sources(n, seed):
    return np.concatenate([np.arange(n), synth.sources(500, n, seed), [-1, n]]).astype(np.int32)


@pytest.mark.parametrize("algo", ["deepwalk", "ppr"])
@pytest.mark.parametrize("sampler", ["naive", "alias", "its", "rej"])
def test_static_programs_equal_builtin_and_oracle(env, algo, sampler):
    case = env["dir" if algo == "ppr" else "sym"]
    g, G = case["g"], case["G"]
    src = _sources(g.n, 5)
    d_src = torch.from_numpy(src).cuda()
    stop = trw.stop_threshold(0.2) if algo == "ppr" else 0
    source = trw.programs.ppr(sampler) if algo == "ppr" else trw.programs.deepwalk(sampler)
    prog = trw.Program(source)
    table = case[sampler] if sampler != "naive" else None
    max_len = 60
    got = _np(*prog.walk(G, table, d_src, max_len, 77, user=(stop,), qid_base=9))
    p = trw.make_params(algo, sampler, max_len, 77, stop_q32=stop)
    ref = _np(*trw.walk(G, table, p, d_src, qid_base=9))
    _same(got, ref, max_len)
    kw = {}
    if sampler == "alias":
        kw = dict(zip(("thr", "alias"), oracle.alias_build(g.row_ptr, g.weight)))
    elif sampler == "its":
        kw = dict(prefix=oracle.its_build(g.row_ptr, g.weight))
    elif sampler == "rej":
        kw = dict(weight=g.weight, pmax=oracle.rej_build(g.row_ptr, g.weight))
    op = oracle.WalkParams(oracle.ALGOS[algo], oracle.SAMPLERS[sampler], max_len, 77, stop_q32=stop)
    orc = oracle.walk(g.row_ptr, g.col, op, src, qid_base=9, **kw)
    _same(got, (orc.paths, orc.lengths, orc.status), max_len)
    prog.close()


@pytest.mark.parametrize("graph", ["sym", "dir"])
@pytest.mark.parametrize("index", [False, True])
def test_node2vec_program_equals_builtin_and_oracle(env, graph, index):
    case = env[graph]
    g, G = case["g"], case["G"]
    src = _sources(g.n, 6)
    d_src = torch.from_numpy(src).cuda()
    prog = trw.Program(trw.programs.NODE2VEC)
    for pq in ((2.0, 0.5), (0.25, 4.0)):
        thr = trw.n2v_thresholds(*pq)
        table = case["eidx"] if index else None
        got = _np(*prog.walk(G, table, d_src, 40, 123, user=thr))
        p = trw.make_params("node2vec", "orej", 40, 123, n2v_thr_q16=thr)
        ref = _np(*trw.walk(G, None, p, d_src))
        _same(got, ref, 40)
        op = oracle.WalkParams(oracle.NODE2VEC, oracle.OREJ, 40, 123, n2v_thr_q16=tuple(thr))
        orc = oracle.walk(g.row_ptr, g.col, op, src)
        _same(got, (orc.paths, orc.lengths, orc.status), 40)
    prog.close()


def test_metapath_program_equals_builtin_and_oracle(env):
    case = env["sym"]
    g, G = case["g"], case["G"]
    src = _sources(g.n, 7)
    d_src = torch.from_numpy(src).cuda()
    schema = (3, 1, 4, 1, 0)
    prog = trw.Program(trw.programs.METAPATH)
    got = _np(*prog.walk(G, None, d_src, 50, 31, user=(len(schema),) + schema))
    p = trw.make_params("metapath", "its", 50, 31, schema=schema)
    ref = _np(*trw.walk(G, None, p, d_src))
    _same(got, ref, 50)
    op = oracle.WalkParams(oracle.METAPATH, oracle.ITS, 50, 31, schema=schema)
    orc = oracle.walk(g.row_ptr, g.col, op, src, label=g.label)
    _same(got, (orc.paths, orc.lengths, orc.status), 50)
    prog.close()


@pytest.mark.parametrize("bound", ["rej_table", "global", "global+eidx"])
@pytest.mark.parametrize("graph", ["sym", "dir"])
def test_weighted_node2vec_program_equals_oracle(env, graph, bound):
    """Weighted Node2Vec (transition weight w(e) times the second-order factor) by rejection:
    a dart hits iff r1 * bound < w * factor * 2^16, exactly, as the oracle's."""
    case = env[graph]
    g, G = case["g"], case["G"]
    assert g.weight.min() >= 1 and g.weight.max() <= 255
    src = _sources(g.n, 8)
    d_src = torch.from_numpy(src).cuda()
    prog = trw.Program(trw.programs.WEIGHTED_NODE2VEC)
    table = {"rej_table": case["rej"], "global": None, "global+eidx": case["eidx"]}[bound]
    pmax = oracle.rej_build(g.row_ptr, g.weight) if bound == "rej_table" else np.full(g.n, 255, np.uint32)
    for pq in ((2.0, 0.5), (0.25, 4.0)):
        thr = trw.n2v_thresholds(*pq)
        got = _np(*prog.walk(G, table, d_src, 40, 321, user=tuple(thr) + (255,), qid_base=1 << 36))
        op = oracle.WalkParams(oracle.NODE2VEC, oracle.REJ, 40, 321, n2v_thr_q16=tuple(thr))
        orc = oracle.walk(g.row_ptr, g.col, op, src, qid_base=1 << 36, weight=g.weight, pmax=pmax)
        _same(got, (orc.paths, orc.lengths, orc.status), 40)
        log(f"  {graph} {bound} p,q={pq}: {int(orc.lengths.sum())} moves identical")
    prog.close()


@pytest.mark.parametrize("index", [False, True])
@pytest.mark.parametrize("graph", ["sym", "dir"])
def test_node2vec_its_program_equals_oracle(env, graph, index):
    """Node2Vec by dynamic ITS (lane scans below 128 slots, wave scans above) against the oracle."""
    case = env[graph]
    g, G = case["g"], case["G"]
    assert g.degrees().max() >= 128
    src = _sources(g.n, 9)
    d_src = torch.from_numpy(src).cuda()
    prog = trw.Program(trw.programs.NODE2VEC_ITS)
    for thr in (trw.n2v_thresholds(2.0, 0.5), (1, 2, 4), (0, 7, 3)):
        got = _np(*prog.walk(G, case["eidx"] if index else None, d_src, 30, 55, user=tuple(thr)))
        op = oracle.WalkParams(oracle.NODE2VEC, oracle.ITS, 30, 55, n2v_thr_q16=tuple(thr))
        orc = oracle.walk(g.row_ptr, g.col, op, src)
        _same(got, (orc.paths, orc.lengths, orc.status), 30)
        log(f"  {graph} thresholds {tuple(thr)}: {int(orc.lengths.sum())} moves identical")
    prog.close()


def test_node2vec_its_program_wide_draw():
    """A hub of 70,000 slots: the first move's total 65536 * d exceeds 2^32, so the draw is the
    high half of (r1:r0) * W (wave scan), as in the oracle."""
    from helpers import star
    g = star(70_000)
    G = trw.Graph(g.row_ptr, g.col, None)
    assert G.validate() == 0
    src = np.concatenate([np.zeros(3000), np.arange(1, 200)]).astype(np.int32)
    prog = trw.Program(trw.programs.NODE2VEC_ITS)
    thr = trw.n2v_thresholds(2.0, 0.5)
    got = _np(*prog.walk(G, None, torch.from_numpy(src).cuda(), 6, 4, user=tuple(thr)))
    orc = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.NODE2VEC, oracle.ITS, 6, 4, n2v_thr_q16=tuple(thr)),
                      src)
    _same(got, (orc.paths, orc.lengths, orc.status), 6)
    assert len(np.unique(got[0][:3000, 1])) > 2500
    prog.close()


@pytest.mark.parametrize("bound", ["rej_table", "global"])
def test_weighted_rej_program_equals_oracle(env, bound):
    """The weighted walk by rejection against the oracle's REJ with the same bound (the row's
    largest weight from a REJ table, or 255 for every row)."""
    case = env["dir"]
    g, G = case["g"], case["G"]
    src = _sources(g.n, 10)
    prog = trw.Program(trw.programs.WEIGHTED_REJ)
    got = _np(*prog.walk(G, case["rej"] if bound == "rej_table" else None, torch.from_numpy(src).cuda(), 50, 66,
                         user=(255,)))
    pmax = oracle.rej_build(g.row_ptr, g.weight) if bound == "rej_table" else np.full(g.n, 255, np.uint32)
    orc = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.DEEPWALK, oracle.REJ, 50, 66), src,
                      weight=g.weight, pmax=pmax)
    _same(got, (orc.paths, orc.lengths, orc.status), 50)
    prog.close()


def test_weighted_node2vec_second_order_law(env):
    """Two-move walks on a small weighted graph: the second move's frequencies
    against the exact law P(x | prev, cur) ~ factor(prev, x) * w(cur, x)."""
    # triangle 0-1-2 with a tail 2-3 and a chord 1-3; a global bound of 255 that divides
    # none of the products factor * w (the acceptance is compared exactly)
    pairs = [(0, 1), (1, 2), (0, 2), (2, 3), (1, 3)]
    weights = [3, 5, 2, 8, 1]
    gt = undirected(4, pairs, weights=weights)
    G = trw.Graph(gt.row_ptr, gt.col, gt.weight, symmetric=True)
    assert G.validate() == 0
    prog = trw.Program(trw.programs.WEIGHTED_NODE2VEC)
    thr = trw.n2v_thresholds(2.0, 0.5)          # 16384, 32768, 65536
    nq = 1 << 20
    d_src = torch.ones(nq, dtype=torch.int32, device="cuda")      # every walk starts at vertex 1
    P, L, S = _np(*prog.walk(G, None, d_src, 2, 2024, user=tuple(thr) + (255,)))
    assert (L == 2).all()
    rp, col, w = gt.row_ptr, gt.col, gt.weight
    adj = {(int(u), int(col[e])): int(w[e]) for u in range(4) for e in range(rp[u], rp[u + 1])}
    for cur in np.unique(P[:, 1]):
        sel = P[:, 1] == cur
        nxt = P[sel, 2]
        cand = [int(x) for x in col[rp[cur]:rp[cur + 1]]]
        expect = []
        for x in cand:
            f = thr[0] if x == 1 else (thr[1] if (1, x) in adj else thr[2])
            expect.append(f * adj[(int(cur), x)])
        expect = np.array(expect, float) / sum(expect)
        counts = np.array([(nxt == x).sum() for x in cand])
        assert counts.sum() == sel.sum()
        if len(cand) > 1:
            stat, pval = scipy.stats.chisquare(counts, expect * counts.sum())
            log(f"  cur={cur} counts={counts.tolist()} p={pval:.3g}")
            assert pval > 1e-6
    prog.close()


def test_program_errors(env):
    case = env["sym"]
    with pytest.raises(trw.TrwError):
        trw.Program(trw.programs.NODE2VEC.replace("return false;", "return undefined_name;"))
    prog = trw.Program(trw.programs.deepwalk("alias"))
    src = torch.arange(10, dtype=torch.int32, device="cuda")
    with pytest.raises(trw.TrwError):          # a STATIC_ALIAS program needs the ALIAS table
        prog.walk(case["G"], None, src, 5, 1)
    with pytest.raises(trw.TrwError):
        prog.walk(case["G"], case["alias"], src, 0, 1)
    prog.close()


def test_metapath_program_on_hub_rows():
    """Rows of 1..6000 labels (lane scans below 128 slots, wave scans above):
    the program equals the built-in walk and the oracle."""
    rng = np.random.default_rng(3)
    edges, labs = [], []
    n = 6500
    for v in range(40):
        d = int(rng.integers(1, 6000)) if v % 3 else int(rng.integers(1, 9))
        nb = np.sort(rng.choice(np.arange(40, n), size=d, replace=False))
        edges += [(v, int(x)) for x in nb]
        labs += rng.integers(0, 4, size=d).tolist()
    for x in range(40, n):
        for h in (0, 1, 2):
            edges.append((x, h))
            labs.append(int(rng.integers(0, 4)))
    g = synth.from_edges(n, edges, labels=labs)
    G = trw.Graph(g.row_ptr, g.col, None, g.label)
    assert G.validate() == 0
    src = np.tile(np.arange(40, dtype=np.int32), 64)
    d_src = torch.from_numpy(src).cuda()
    schema = (1, 0, 3, 2)
    prog = trw.Program(trw.programs.METAPATH)
    got = _np(*prog.walk(G, None, d_src, 30, 17, user=(len(schema),) + schema))
    ref = _np(*trw.walk(G, None, trw.make_params("metapath", "its", 30, 17, schema=schema), d_src))
    _same(got, ref, 30)
    orc = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.METAPATH, oracle.ITS, 30, 17, schema=schema), src,
                      label=g.label)
    _same(got, (orc.paths, orc.lengths, orc.status), 30)
    prog.close()


def _second_move_law(P, cur_first, expect_fn):
    """χ² of the second move's destination for each first-move vertex."""
    for cur in np.unique(P[:, 1]):
        sel = P[:, 1] == cur
        nxt = P[sel, 2]
        cand, expect = expect_fn(int(cur))
        counts = np.array([(nxt == x).sum() for x in cand])
        assert counts.sum() == sel.sum()
        if len(cand) > 1:
            _, pval = scipy.stats.chisquare(counts, np.array(expect, float) / sum(expect) * counts.sum())
            log(f"  cur={cur} counts={counts.tolist()} p={pval:.3g}")
            assert pval > 1e-6


def test_node2vec_its_program_law():
    """Node2Vec by dynamic ITS: P(x | prev, cur) proportional to the factor of x."""
    pairs = [(0, 1), (1, 2), (0, 2), (2, 3), (1, 3)]
    gt = undirected(4, pairs)
    G = trw.Graph(gt.row_ptr, gt.col, None, symmetric=True)
    assert G.validate() == 0
    prog = trw.Program(trw.programs.NODE2VEC_ITS)
    f = (1, 2, 4)                                   # 1/p, 1, 1/q for p = 2, q = 0.5, as integers
    d_src = torch.ones(1 << 20, dtype=torch.int32, device="cuda")
    P, L, S = _np(*prog.walk(G, None, d_src, 2, 99, user=f))
    assert (L == 2).all()
    rp, col = gt.row_ptr, gt.col
    nb = {u: set(int(x) for x in col[rp[u]:rp[u + 1]]) for u in range(4)}
    first = np.bincount(P[:, 1], minlength=4)[sorted(nb[1])]
    _, pval = scipy.stats.chisquare(first)              # first move uniform
    assert pval > 1e-6

    def expect(cur):
        cand = sorted(nb[cur])
        return cand, [f[0] if x == 1 else (f[1] if x in nb[1] else f[2]) for x in cand]
    _second_move_law(P, 1, expect)
    prog.close()


def test_weighted_rej_program_law():
    """REJ with a global bound: each move follows e with probability w(e) / sum of the row."""
    gt = synth.from_edges(5, [(0, 1), (0, 2), (0, 3), (0, 4), (1, 0), (2, 0), (3, 0), (4, 0)],
                          weights=[1, 2, 3, 10, 1, 1, 1, 1])
    G = trw.Graph(gt.row_ptr, gt.col, gt.weight)
    assert G.validate() == 0
    prog = trw.Program(trw.programs.WEIGHTED_REJ)
    d_src = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
    P, L, S = _np(*prog.walk(G, None, d_src, 1, 5, user=(255,)))    # 255 bounds every weight
    assert (L == 1).all()
    counts = np.bincount(P[:, 1], minlength=5)[1:]
    _, pval = scipy.stats.chisquare(counts, np.array([1, 2, 3, 10]) / 16 * counts.sum())
    log(f"  counts={counts.tolist()} p={pval:.3g}")
    assert pval > 1e-6
    prog.close()
