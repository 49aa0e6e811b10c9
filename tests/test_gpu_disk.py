"""Walks over a graph kept in a file, vertex-range partitions loaded onto the
device as the walks need them (trw_disk_walk): every query's path, length and
status equal the oracle's on the whole graph, for every supported (algorithm,
sampler), with many partitions, hub rows alone in theirs, one partition, and
one, a few or all partitions resident at once."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

trw = pytest.importorskip("paper_2107_11983_amd")


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def graph(tmp_path_factory):
    g = synth.rmat(12, 16, False, 0xD15C)
    synth.attach_attrs(g, 0xD15C ^ 3, weights=True, labels=4)
    path = str(tmp_path_factory.mktemp("disk") / "g.csr")
    trw.write_disk_graph(path, g.row_ptr.astype(np.int64), g.col, g.weight, g.label)
    return g, path


CASES = [("deepwalk", "naive", 40), ("deepwalk", "alias", 40), ("deepwalk", "its", 40), ("deepwalk", "rej", 40),
         ("ppr", "naive", 64), ("ppr", "alias", 64), ("ppr", "its", 64), ("ppr", "rej", 64),
         ("metapath", "its", 20), ("node2vec", "orej", 30)]
SCHEMA = (0, 1, 2, 1)
N2V_THR = (16384, 32768, 65536)     # p = 2, q = 0.5


def params(algo, sampler, max_len, seed):
    kw = {}
    if algo == "ppr":
        kw["stop_q32"] = trw.stop_threshold(0.15)
    if algo == "metapath":
        kw["schema"] = SCHEMA
    if algo == "node2vec":
        kw["n2v_thr_q16"] = N2V_THR
    return trw.make_params(algo, sampler, max_len, seed, **kw)


def oracle_walk(g, algo, sampler, max_len, seed, src, qid_base, stop):
    op = oracle.WalkParams(oracle.ALGOS[algo], oracle.SAMPLERS[sampler], max_len, seed, stop_q32=stop,
                           schema=SCHEMA if algo == "metapath" else (),
                           n2v_thr_q16=N2V_THR if algo == "node2vec" else (65536, 65536, 65536))
    kw = {}
    if algo == "metapath":
        kw["label"] = g.label
    elif sampler == "alias":
        kw["thr"], kw["alias"] = oracle.alias_build(g.row_ptr, g.weight)
    elif sampler == "its":
        kw["prefix"] = oracle.its_build(g.row_ptr, g.weight)
    elif sampler == "rej":
        kw["weight"], kw["pmax"] = g.weight, oracle.rej_build(g.row_ptr, g.weight)
    return oracle.walk(g.row_ptr, g.col, op, src, qid_base=qid_base, **kw)


def same_as(ref, P, L, S, max_len):
    P, L, S = P.cpu().numpy(), L.cpu().numpy().view(np.uint32), S.cpu().numpy()
    assert np.array_equal(S, ref.status)
    assert np.array_equal(L, ref.lengths)
    ok = ref.status != oracle.ST_BAD_SOURCE
    mask = (np.arange(max_len + 1)[None, :] <= ref.lengths[:, None]) & ok[:, None]
    assert np.array_equal(P[:, :max_len + 1][mask], ref.paths[mask])


def part_sizes(g):
    deg = np.diff(g.row_ptr.astype(np.int64))
    return {"sevenths": g.m // 7, "hubs_alone": int(deg.max()) // 2, "one": 0}


@pytest.mark.parametrize("split,slots", [("sevenths", 1), ("sevenths", 3), ("sevenths", 99), ("hubs_alone", 1),
                                         ("hubs_alone", 16), ("one", 1)])
@pytest.mark.parametrize("algo,sampler,max_len", CASES)
def test_disk_walk_equals_oracle(graph, algo, sampler, max_len, split, slots):
    g, path = graph
    pe = part_sizes(g)[split]
    G = trw.DiskGraph(path, pe)
    src = np.concatenate([synth.sources(3000, g.n, 41), np.array([-1, g.n], np.int32)]).astype(np.int32)
    p = params(algo, sampler, max_len, 1234)
    log(f"  disk {algo}/{sampler} part_edges={pe} parts={G.parts} slots={slots} nq={len(src)}")
    P, L, S, st = G.walk(p, torch.from_numpy(src).cuda(), qid_base=77, slots=slots)
    torch.cuda.synchronize()
    ref = oracle_walk(g, algo, sampler, max_len, 1234, src, 77, int(p.stop_q32))
    same_as(ref, P, L, S, max_len)
    # a round loads at most one partition (Node2Vec: the two of a pair)
    assert 1 <= st["loads"] <= (2 if algo == "node2vec" else 1) * st["runs"]
    per_edge = 4 + (4 if sampler in ("alias", "its", "rej") and algo != "metapath" else 0) + \
        (1 if algo == "metapath" else 0)
    sizes = [G.partition(i)[3] - G.partition(i)[2] for i in range(G.parts)]
    if slots == 1 and algo != "node2vec":
        assert st["loads"] == st["runs"]          # the partition just walked holds no waiting query
    if slots >= G.parts:
        # nothing is evicted: each partition is read at most once
        assert st["loads"] <= G.parts and st["bytes_read"] <= g.m * per_edge
    if G.parts == 1:
        assert st["runs"] == 1 and st["loads"] == 1 and st["bytes_read"] == g.m * per_edge
    else:
        assert st["bytes_read"] >= per_edge * min(sizes)
    G.close()


def test_disk_walk_equals_in_memory_walk(graph):
    """The same queries through trw_walk on the whole graph in device memory."""
    g, path = graph
    G = trw.DiskGraph(path, g.m // 5)
    Gm = trw.Graph(g.row_ptr, g.col, g.weight)
    alias = Gm.table("alias")
    src = synth.sources(20000, g.n, 5)
    p = params("deepwalk", "alias", 80, 99)
    qid_base = (1 << 40) + 5
    P, L, S, st = G.walk(p, torch.from_numpy(src).cuda(), qid_base=qid_base, slots=2)
    P2, L2, S2 = trw.walk(Gm, alias, p, torch.from_numpy(src).cuda(), qid_base=qid_base)
    torch.cuda.synchronize()
    assert torch.equal(L, L2) and torch.equal(S, S2)
    mask = torch.arange(81, device=P.device)[None, :] <= L[:, None]
    assert torch.equal(P[mask], P2[:, :81][mask])
    log(f"  runs={st['runs']} loads={st['loads']} read={st['bytes_read']} B")
    Gm.close()
    G.close()


def test_disk_walk_edge_cases(graph, tmp_path):
    g, path = graph
    G = trw.DiskGraph(path, g.m // 3)
    # one query, max_len 1; a batch of bad sources only; a wide output row
    for src, max_len, stride in ((np.array([5], np.int32), 1, None), (np.array([-7, g.n, 1 << 30], np.int32), 5, None),
                                 (synth.sources(513, g.n, 8), 7, 19)):
        p = params("ppr", "naive", max_len, 3)
        P, L, S, _ = G.walk(p, torch.from_numpy(src).cuda(), stride=stride, slots=2)
        torch.cuda.synchronize()
        ref = oracle_walk(g, "ppr", "naive", max_len, 3, src, 0, int(p.stop_q32))
        same_as(ref, P, L, S, max_len)
    # an empty batch
    P, L, S, st = G.walk(params("deepwalk", "naive", 5, 3), torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert P.shape[0] == 0 and st["runs"] == 0
    G.close()


def test_destination_out_of_range_is_refused(graph, tmp_path):
    """A file whose partition holds an edge to a vertex >= n: the load checks the
    destinations on the host and the walk fails with TRW_E_INVALID."""
    g, _ = graph
    col = g.col.copy()
    bad_v = int(np.argmax(np.diff(g.row_ptr)))          # the largest row, so the first load holds it
    col[g.row_ptr[bad_v]] = g.n
    path = str(tmp_path / "bad.csr")
    trw.write_disk_graph(path, g.row_ptr.astype(np.int64), col, g.weight)
    G = trw.DiskGraph(path, g.m // 4)
    src = np.full(64, bad_v, np.int32)
    with pytest.raises(trw.TrwError, match="outside"):
        G.walk(params("deepwalk", "naive", 10, 1), torch.from_numpy(src).cuda())
    G.close()


@pytest.mark.parametrize("split,slots", [("sevenths", 2), ("sevenths", 99), ("hubs_alone", 4)])
def test_disk_node2vec_symmetric(tmp_path, split, slots):
    """Node2Vec on a symmetric graph (a move often returns to the previous vertex's
    partition): every query equals the oracle's."""
    g = synth.rmat(12, 16, True, 0x5E7)
    path = str(tmp_path / "sym.csr")
    trw.write_disk_graph(path, g.row_ptr.astype(np.int64), g.col)
    G = trw.DiskGraph(path, part_sizes(g)[split])
    src = synth.sources(4000, g.n, 17)
    p = params("node2vec", "orej", 40, 555)
    log(f"  disk node2vec symmetric parts={G.parts} slots={slots}")
    P, L, S, st = G.walk(p, torch.from_numpy(src).cuda(), qid_base=9, slots=slots)
    torch.cuda.synchronize()
    ref = oracle_walk(g, "node2vec", "orej", 40, 555, src, 9, 0)
    same_as(ref, P, L, S, 40)
    log(f"  runs={st['runs']} loads={st['loads']}")
    G.close()


def test_disk_node2vec_needs_sorted_rows(graph, tmp_path):
    """Node2Vec searches the previous vertex's row: a partition with an unsorted row is
    refused when it is loaded (a host check; the other walks take such rows)."""
    g, _ = graph
    col = g.col.copy()
    v = int(np.argmax(np.diff(g.row_ptr)))
    a, b = int(g.row_ptr[v]), int(g.row_ptr[v + 1])
    col[a:b] = col[a:b][::-1]
    path = str(tmp_path / "unsorted.csr")
    trw.write_disk_graph(path, g.row_ptr.astype(np.int64), col)
    G = trw.DiskGraph(path, g.m // 4)
    src = np.full(32, v, np.int32)
    with pytest.raises(trw.TrwError, match="not sorted"):
        G.walk(params("node2vec", "orej", 10, 1), torch.from_numpy(src).cuda(), slots=2)
    P, L, S, _ = G.walk(params("deepwalk", "naive", 10, 1), torch.from_numpy(src).cuda(), slots=2)
    torch.cuda.synchronize()
    assert (S.cpu().numpy() != 0).all()
    G.close()


def test_disk_walk_on_a_side_stream(graph):
    """The walk launched on a stream of its own (default priority) gives the same
    outputs as on the current stream."""
    g, path = graph
    G = trw.DiskGraph(path, g.m // 5)
    src = torch.from_numpy(synth.sources(5000, g.n, 23)).cuda()
    p = params("ppr", "its", 64, 31)
    P0, L0, S0, _ = G.walk(p, src, qid_base=3, slots=2)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        P1, L1, S1, st = G.walk(p, src, qid_base=3, slots=2, stream=s)
    s.synchronize()
    assert torch.equal(L0, L1) and torch.equal(S0, S1)
    mask = torch.arange(P0.shape[1], device=P0.device)[None, :] <= L0[:, None]
    assert torch.equal(P0[mask], P1[mask])
    assert st["runs"] >= 1
    G.close()
