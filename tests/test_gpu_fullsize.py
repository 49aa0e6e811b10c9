"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (persistent schedule, default tuning, the same tables and indexes).

* PPR on R-MAT 2^22 (10^7 queries): every query compared with the oracle,
  paths included, in chunks of 10^6; the end counts of five groups of
  2 M queries and their top 4096 compared whole, also from the counting
  walk that writes no paths; the same batch with REJ
  compared on a seeded sample.
* Node2Vec and MetaPath on R-MAT 2^24 (one query per vertex): a seeded sample
  of queries compared with the oracle, which walks exactly those query ids;
  the termination rules checked on every query and the hops of a sample
  checked against the CSR rows.
* The served mix on R-MAT 2^26 (about 1.07 G directed edges): requests of
  every algorithm through the server, a sample of each compared with the
  oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

trw = None


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    global trw
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2107_11983_amd as mod
    trw = mod
    torch.cuda.set_device(0)
    yield
    torch.cuda.empty_cache()


def _params(wl, sampler):
    kw = {}
    if wl.algo == "ppr":
        kw["stop_q32"] = trw.stop_threshold(wl.stop_prob)
    if wl.algo == "node2vec":
        kw["n2v_thr_q16"] = trw.n2v_thresholds(*wl.n2v_pq)
    if wl.algo == "metapath":
        kw["schema"] = [int(x) for x in synth.make_schema(wl)]
    return trw.make_params(wl.algo, sampler, wl.max_len, wl.walk_seed, **kw)


def _oracle_params(p):
    algo = {v: k for k, v in trw.ALGOS.items()}[int(p.algo)]
    sampler = {v: k for k, v in trw.SAMPLERS.items()}[int(p.sampler)]
    return oracle.WalkParams(oracle.ALGOS[algo], oracle.SAMPLERS[sampler], int(p.max_len), int(p.seed),
                             stop_q32=int(p.stop_q32),
                             n2v_thr_q16=tuple(int(x) for x in p.n2v_thr_q16),
                             schema=tuple(int(p.schema[i]) for i in range(p.schema_len)))


def _rows(t, idx):
    """Rows idx of a device tensor, on the host."""
    return t[torch.from_numpy(idx).to(t.device)].cpu().numpy()


def _compare(P, L, S, ref, max_len, what):
    L = L.view(np.uint32) if L.dtype != np.uint32 else L
    bad = np.nonzero((L != ref.lengths) | (S != ref.status))[0]
    assert bad.size == 0, f"{what}: lengths/status differ at {bad[:8]}"
    mask = np.arange(max_len + 1)[None, :] <= ref.lengths[:, None]
    diff = np.nonzero(((P[:, :max_len + 1] != ref.paths) & mask).any(axis=1))[0]
    assert diff.size == 0, f"{what}: paths differ at {diff[:8]}"


def _check_rules(wl, L, S):
    """Termination rules on every query (lengths, status)."""
    L = L.view(np.uint32)
    assert set(np.unique(S).tolist()) <= {1, 2, 3}
    assert (L <= wl.max_len).all()
    full = S == 1
    assert (L[full] == wl.max_len).all()
    if wl.algo == "ppr":
        assert ((L[S == 2] >= 1)).all()
    else:
        assert not (S == 2).any()


def _check_hops(g, P, L):
    """Every hop of the sampled paths is an edge of the CSR graph."""
    rp = g.row_ptr.astype(np.int64)
    for i in range(P.shape[0]):
        for k in range(int(L[i])):
            u, v = int(P[i, k]), int(P[i, k + 1])
            row = g.col[rp[u]:rp[u + 1]]
            j = np.searchsorted(row, v)
            assert j < row.size and row[j] == v, f"hop {u}->{v} is not an edge"


def _walk_full(wl, G, table, p, src):
    d_src = torch.from_numpy(src).cuda()
    P, L, S = trw.walk(G, table, p, d_src)      # persistent, default tuning (as timed by bench.py)
    torch.cuda.synchronize()
    return P, L, S


def test_ppr_rmat22_every_query():
    wl = synth.WORKLOADS["ppr-rmat22"]
    g = synth.make_graph(wl)
    src = synth.make_sources(wl, g)
    log(f"  ppr-rmat22: n={g.n} m={g.m} nq={len(src)}")
    G = trw.Graph(g.row_ptr, g.col, g.weight, symmetric=wl.symmetric)
    assert G.validate() == 0
    alias = G.table("alias")
    p = _params(wl, "alias")
    P, L, S = _walk_full(wl, G, alias, p, src)
    Lh, Sh = L.cpu().numpy(), S.cpu().numpy()
    _check_rules(wl, Lh, Sh)
    thr, al = oracle.alias_build(g.row_ptr, g.weight)
    op = _oracle_params(p)
    chunk = 1_000_000
    group = 2_000_000
    exp_counts = np.zeros((len(src) // group, g.n), np.uint32)
    for lo in range(0, len(src), chunk):
        hi = min(len(src), lo + chunk)
        ref = oracle.walk(g.row_ptr, g.col, op, src[lo:hi], qid_base=lo, thr=thr, alias=al)
        Pc = P[lo:hi].cpu().numpy()
        _compare(Pc, Lh[lo:hi], Sh[lo:hi], ref, wl.max_len, f"ppr-rmat22 queries {lo}..{hi}")
        log(f"  ppr-rmat22 queries {lo}..{hi} identical")
        # the oracle's end counts of the same queries (groups of 2 M queries hold whole chunks)
        oracle.end_counts(g.n, ref.paths, ref.lengths, ref.status, counts=exp_counts[lo // group])
    # PPR estimate at full size: end counts per group and the top 4096 of each group
    counts, skipped = trw.ppr_end_counts(G, P, L, S, group=group)
    torch.cuda.synchronize()
    assert int(skipped.item()) == 0
    got = counts.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, exp_counts), "end counts differ"
    for gi in range(exp_counts.shape[0]):
        ids, vals = trw.topk(counts[gi], 4096)
        eid, ev = oracle.topk(exp_counts[gi], 4096)
        assert np.array_equal(ids.cpu().numpy(), eid) and np.array_equal(vals.cpu().numpy().view(np.uint32), ev)
    log("  ppr-rmat22 end counts and top-4096 identical")
    del counts, P, L, S
    # the counting walk (no paths) gives the same counts, lengths and status
    counts, L2, S2 = trw.ppr_walk_counts(G, alias, p, torch.from_numpy(src).cuda(), group=group)
    torch.cuda.synchronize()
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), exp_counts), "counting walk differs"
    assert np.array_equal(L2.cpu().numpy(), Lh) and np.array_equal(S2.cpu().numpy(), Sh)
    log("  ppr-rmat22 counting walk identical")
    del counts, L2, S2
    # REJ on the same batch: a seeded sample of queries against the oracle
    rej = G.table("rej")
    pr = _params(wl, "rej")
    P, L, S = _walk_full(wl, G, rej, pr, src)
    Lh, Sh = L.cpu().numpy(), S.cpu().numpy()
    _check_rules(wl, Lh, Sh)
    idx = np.unique(np.concatenate([np.random.default_rng(7).choice(len(src), 20000, replace=False),
                                    [0, len(src) - 1]]))
    ref = oracle.walk(g.row_ptr, g.col, _oracle_params(pr), src[idx], qids=idx.astype(np.uint64),
                      weight=g.weight, pmax=oracle.rej_build(g.row_ptr, g.weight))
    _compare(_rows(P, idx), Lh[idx], Sh[idx], ref, wl.max_len, "ppr-rmat22 REJ sample")
    log("  ppr-rmat22 REJ sample identical")
    G.close()


@pytest.mark.parametrize("name,sampler,index", [("node2vec-rmat24", "orej", "edge"),
                                                ("metapath-rmat24", "its", "label")])
def test_rmat24_sampled_queries(name, sampler, index):
    wl = synth.WORKLOADS[name]
    g = synth.make_graph(wl)
    src = synth.make_sources(wl, g)
    log(f"  {name}: n={g.n} m={g.m} nq={len(src)}")
    G = trw.Graph(g.row_ptr, g.col, g.weight, g.label, symmetric=wl.symmetric)
    assert G.validate() == 0
    table = G.edge_index() if index == "edge" else G.label_index(wl.labels)
    p = _params(wl, sampler)
    P, L, S = _walk_full(wl, G, table, p, src)
    Lh, Sh = L.cpu().numpy(), S.cpu().numpy()
    _check_rules(wl, Lh, Sh)
    rng = np.random.default_rng(2024)
    n_sample = 20000 if wl.algo == "node2vec" else 6000
    idx = np.sort(rng.choice(len(src), size=n_sample, replace=False))
    idx = np.unique(np.concatenate([idx, [0, len(src) - 1]]))     # the first and last query too
    ref = oracle.walk(g.row_ptr, g.col, _oracle_params(p), src[idx], qids=idx.astype(np.uint64),
                      label=g.label if wl.algo == "metapath" else None)
    Ps = _rows(P, idx)
    _compare(Ps, Lh[idx], Sh[idx], ref, wl.max_len, name)
    _check_hops(g, Ps[:300], Lh[idx][:300].view(np.uint32))
    log(f"  {name}: {idx.size} sampled queries identical, rules hold for all {len(src)}")
    G.close()


def test_served_rmat26_sampled_queries():
    wl = synth.WORKLOADS["served-rmat26"]
    g = synth.make_graph(wl)
    log(f"  served-rmat26: n={g.n} m={g.m}")
    G = trw.Graph(g.row_ptr, g.col, g.weight, symmetric=True)
    assert G.validate() == 0
    alias = G.table("alias")
    eidx = G.edge_index()
    srv = trw.Server(G, alias, eidx, pool_bytes=2 << 30)
    rng = np.random.default_rng(77)
    algos = [("deepwalk", "alias", 80), ("ppr", "alias", 256), ("node2vec", "orej", 80)]
    reqs = []
    for r in range(12):
        algo, sampler, max_len = algos[r % 3]
        nq = int(rng.integers(1, 4097))
        src = synth.sources(nq, g.n, 0x5AC0000005 + r)
        kw = {}
        if algo == "ppr":
            kw["stop_q32"] = trw.stop_threshold(0.2)
        if algo == "node2vec":
            kw["n2v_thr_q16"] = trw.n2v_thresholds(2.0, 0.5)
        p = trw.make_params(algo, sampler, max_len, wl.walk_seed + r, **kw)
        rid = srv.submit(p, src, qid_base=(r + 1) << 32)
        reqs.append((rid, p, src, (r + 1) << 32))
    got = {}
    import time
    t0 = time.time()
    while len(got) < len(reqs):
        assert time.time() - t0 < 60, "served requests did not complete"
        for c in srv.poll(64, timeout_ms=100):
            got[c["request_id"]] = c
    thr, al = oracle.alias_build(g.row_ptr, g.weight)
    for rid, p, src, qb in reqs:
        c = got[rid]
        assert c["status"] == 0
        nq = len(src)
        idx = np.unique(np.concatenate([rng.choice(nq, size=min(nq, 200), replace=False), [0, nq - 1]]))
        kw = dict(thr=thr, alias=al) if int(p.sampler) == trw.SAMPLERS["alias"] else {}
        ref = oracle.walk(g.row_ptr, g.col, _oracle_params(p), src[idx], qids=(qb + idx).astype(np.uint64), **kw)
        Pd, Ld, Sd = c["paths"], c["lengths"], c["status_codes"]
        Ps = _rows(Pd, idx) if isinstance(Pd, torch.Tensor) else Pd[idx]
        Ls = (_rows(Ld, idx) if isinstance(Ld, torch.Tensor) else Ld[idx]).view(np.uint32)
        Ss = _rows(Sd, idx) if isinstance(Sd, torch.Tensor) else Sd[idx]
        _compare(Ps, Ls, Ss, ref, int(p.max_len), f"served request {rid}")
    log(f"  served-rmat26: {len(reqs)} requests, sampled queries identical")
    srv.close()
    G.close()
