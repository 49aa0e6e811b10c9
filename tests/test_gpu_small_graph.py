"""Walks with the whole graph in LDS (NAIVE DeepWalk and PPR, persistent schedule).

A graph whose CSR fits one workgroup's LDS (int32 row offsets and uint16
destinations, 160 KiB on gfx950) is walked from LDS by default.  Every case
runs twice, with the default and with no_lds_graph set (the general
persistent kernel), and both must equal the oracle bit for bit.  Cases:
dead ends and bad sources, the c1-shaped DeepWalk graph, PPR at several stop
probabilities, graphs exactly at the LDS limit and one edge over it, one
query, a source without out-edges, max_len 1, a wide path stride, a query-id
offset, and a large batch on a small graph.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

trw = None
LDS_LIMIT = 160 * 1024


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    global trw
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2107_11983_amd as mod
    trw = mod
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def log(msg):
    print(msg, flush=True)


def _lds_bytes(n, m):
    r16 = lambda b: (b + 15) // 16 * 16
    return r16(4 * (n + 1)) + r16(2 * m)


def _graph_with_m(n, m, seed):
    """A directed graph on n vertices with exactly m edges, rows sorted, no duplicates or self-loops."""
    rng = np.random.default_rng(seed)
    deg = np.full(n, m // n, np.int64)
    deg[: m - int(deg.sum())] += 1
    rows = []
    for v, d in enumerate(deg):
        t = rng.choice(n - 1, size=int(d), replace=False)
        rows.append(np.sort(t + (t >= v)))
    col = np.concatenate(rows).astype(np.int32)
    row_ptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    assert row_ptr[-1] == m
    return synth.CSRGraph(n, row_ptr, col)


def _both(g, algo, max_len, seed, src, stop=0, qid_base=0, stride=0):
    G = trw.Graph(g.row_ptr, g.col)
    assert G.validate() == 0
    p = trw.make_params(algo, "naive", max_len, seed, stop_q32=stop)
    d_src = torch.from_numpy(np.ascontiguousarray(src, np.int32)).cuda()
    outs = []
    for no_lds in (0, 1):
        bufs = trw.WalkBuffers(G, p, len(src), trw.TRW_M_PERSISTENT, stride)
        bufs.paths.fill_(-7)
        tu = trw.make_tuning(no_lds_graph=1) if no_lds else None
        trw.walk(G, None, p, d_src, qid_base=qid_base, tuning=tu, bufs=bufs)
        torch.cuda.synchronize()
        outs.append((bufs.paths.cpu().numpy(), bufs.lengths.cpu().numpy().view(np.uint32),
                     bufs.status.cpu().numpy()))
    G.close()
    return outs


def _check(out, ref, max_len):
    gp, gl, gs = out
    assert np.array_equal(gs, ref.status)
    assert np.array_equal(gl, ref.lengths)
    ok = ref.status != oracle.ST_BAD_SOURCE
    mask = (np.arange(max_len + 1)[None, :] <= ref.lengths[:, None]) & ok[:, None]
    assert not ((gp[:, :max_len + 1] != ref.paths) & mask).any()
    if (~ok).any():
        assert (gp[~ok] == -7).all()


def _run(g, algo, max_len, seed, src, stop=0, qid_base=0, stride=0):
    lds, plain = _both(g, algo, max_len, seed, src, stop, qid_base, stride)
    ref = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(getattr(oracle, algo.upper()), oracle.NAIVE, max_len, seed,
                                                          stop_q32=stop), np.asarray(src, np.int32), qid_base=qid_base)
    _check(lds, ref, max_len)
    _check(plain, ref, max_len)
    return ref


@pytest.mark.parametrize("algo", ["deepwalk", "ppr"])
def test_dead_ends_and_bad_sources(algo):
    g = synth.from_edges(7, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (5, 6), (6, 5)])   # 4 is a sink
    src = np.array([0, 1, 2, 3, 4, 5, 6, -1, 7, 2, 3] * 37, np.int32)
    log(f"  small graph {algo}: dead ends, bad sources, nq={len(src)}")
    ref = _run(g, algo, 30, 5, src, stop=oracle.stop_q32(0.1) if algo == "ppr" else 0)
    assert (ref.status == oracle.ST_DEAD_END).any() and (ref.status == oracle.ST_BAD_SOURCE).any()


def test_deepwalk_c1_shape():
    """The DeepWalk configuration's graph: symmetric R-MAT, 2^12 vertices, degree 16, q = v."""
    g = synth.rmat(12, 16, True, 0x5A11)
    assert _lds_bytes(g.n, g.m) <= LDS_LIMIT
    for nq in (g.n, g.n + 3, 1, 63):
        src = np.arange(nq, dtype=np.int32) % g.n
        log(f"  small graph deepwalk rmat12 nq={nq}")
        _run(g, "deepwalk", 80, 0x5EED0001, src)


@pytest.mark.parametrize("prob", [0.05, 0.2, 0.9])
def test_ppr_stop_probabilities(prob):
    g = synth.rmat(11, 12, False, 0x5A12)
    src = synth.sources(20001, g.n, 11)
    log(f"  small graph ppr stop={prob}")
    _run(g, "ppr", 256, 77, src, stop=oracle.stop_q32(prob), qid_base=1 << 33)


@pytest.mark.parametrize("extra", [0, 1])
def test_lds_limit(extra):
    """Exactly at the 160 KiB limit (the LDS path) and one edge over it (the general kernel)."""
    n = 4095                                  # row offsets: 16384 bytes
    m = (LDS_LIMIT - 16384) // 2 + extra      # destinations: the rest, or 16 bytes more
    assert (_lds_bytes(n, m) <= LDS_LIMIT) == (extra == 0)
    g = _graph_with_m(n, m, 0x5A13 + extra)
    src = synth.sources(5000, n, 13)
    log(f"  small graph at the LDS limit: n={n} m={m} bytes={_lds_bytes(n, m)}")
    _run(g, "deepwalk", 40, 3, src)
    _run(g, "ppr", 100, 4, src, stop=oracle.stop_q32(0.2))


def test_degenerate_shapes():
    sink = synth.from_edges(2, [(0, 1)])
    log("  small graph: a sink source (length 0) and one move into it")
    ref = _run(sink, "deepwalk", 5, 1, np.array([1] * 70 + [0] * 3, np.int32))
    assert (ref.status == oracle.ST_DEAD_END).all()
    assert (ref.lengths[:70] == 0).all() and (ref.lengths[70:] == 1).all()
    loop = synth.from_edges(2, [(0, 1), (1, 0)])
    log("  small graph: max_len 1, wide stride")
    _run(loop, "deepwalk", 1, 2, np.array([0, 1, 1, 0, 5], np.int32), stride=64)
    _run(loop, "ppr", 1, 2, np.array([0, 1] * 100, np.int32), stop=oracle.stop_q32(0.5))


def test_large_batch_on_small_graph():
    """10^6 PPR queries: 1024-lane workgroups on every CU; the two paths agree on every query and the
    oracle checks the first 20000."""
    g = synth.rmat(12, 16, False, 0x5A14)
    nq = 1_000_000
    src = synth.sources(nq, g.n, 14)
    stop = oracle.stop_q32(0.15)
    log(f"  small graph ppr nq={nq}")
    lds, plain = _both(g, "ppr", 256, 8, src, stop)
    for a, b in zip(lds[1:], plain[1:]):
        assert np.array_equal(a, b)
    L = lds[1].astype(np.int64)
    mask = np.arange(257)[None, :] <= L[:, None]
    assert np.array_equal(np.where(mask, lds[0][:, :257], 0), np.where(mask, plain[0][:, :257], 0))
    ref = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.PPR, oracle.NAIVE, 256, 8, stop_q32=stop), src[:20000])
    _check(tuple(x[:20000] for x in lds), ref, 256)
