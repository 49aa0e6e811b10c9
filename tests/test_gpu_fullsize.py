"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (persistent schedule, default tuning, the same tables and indexes).
Every query of every configuration is compared with the oracle, paths
included; the oracle runs over query ranges on the host's threads (ctypes
releases the interpreter lock while it walks), and the GPU outputs are copied
back in chunks of 2^20 queries.

* PPR on R-MAT 2^22 (10^7 queries) with ALIAS: every query; the end counts of
  five groups of 2 M queries and their top 4096 compared whole, also from the
  counting walk that writes no paths.  The same batch with REJ: every query.
* Node2Vec on R-MAT 2^24 (one query per vertex) with the edge index: every
  query.
* The same Node2Vec batch walked from a CSR file (8 partitions, 4 resident),
  and the PPR batch from a file with ITS and with REJ (17 partitions, 8
  resident): every query equals the in-memory walk.
* MetaPath on R-MAT 2^24 (one query per vertex): every query, once through
  the label index and once by row scans (no index).
* The served mix on R-MAT 2^26 (about 1.06 G directed edges): the bench's
  first replay of 2000 requests submitted at once (saturated), every query of
  every request.
"""
import concurrent.futures
import os
import time

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

trw = None
CHUNK = 1 << 20
WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))


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
    """Every hop of the given paths is an edge of the CSR graph."""
    rp = g.row_ptr.astype(np.int64)
    for i in range(P.shape[0]):
        for k in range(int(L[i])):
            u, v = int(P[i, k]), int(P[i, k + 1])
            row = g.col[rp[u]:rp[u + 1]]
            j = np.searchsorted(row, v)
            assert j < row.size and row[j] == v, f"hop {u}->{v} is not an edge"


class _Merged:
    """Oracle results of consecutive query ranges, joined."""

    def __init__(self, parts):
        self.paths = np.concatenate([r.paths for r in parts])
        self.lengths = np.concatenate([r.lengths for r in parts])
        self.status = np.concatenate([r.status for r in parts])
        self.counters = {}
        for r in parts:
            for k, v in r.counters.items():
                self.counters[k] = self.counters.get(k, 0) + int(v)


def _oracle_range(g, op, src, lo, hi, **tables):
    """The oracle on queries [lo, hi) (ids lo..hi-1), split over the host's threads."""
    step = max(1, -(-(hi - lo) // WORKERS))
    ranges = [(a, min(hi, a + step)) for a in range(lo, hi, step)]

    def run(r):
        return oracle.walk(g.row_ptr, g.col, op, src[r[0]:r[1]], qid_base=r[0], **tables)
    with concurrent.futures.ThreadPoolExecutor(max_workers=WORKERS) as ex:
        return _Merged(list(ex.map(run, ranges)))


def _every_query(name, g, src, outputs, op, max_len, **tables):
    """Compare every query of each (paths, lengths, status) output (device tensors) with the
    oracle, chunk by chunk (the oracle walks each chunk once); returns the oracle's counters."""
    counters = {}
    t0 = time.time()
    for lo in range(0, len(src), CHUNK):
        hi = min(len(src), lo + CHUNK)
        ref = _oracle_range(g, op, src, lo, hi, **tables)
        for j, (P, L, S) in enumerate(outputs):
            _compare(P[lo:hi].cpu().numpy(), L[lo:hi].cpu().numpy(), S[lo:hi].cpu().numpy(), ref, max_len,
                     f"{name} (output {j}) queries {lo}..{hi}")
        for k, v in ref.counters.items():
            counters[k] = counters.get(k, 0) + v
        del ref
    log(f"  {name}: every query identical ({len(src)} queries, {counters.get('moves', 0)} moves, "
        f"{len(outputs)} output(s), oracle on {WORKERS} threads {time.time() - t0:.1f}s)")
    return counters


def _walk_full(G, table, p, src):
    d_src = torch.from_numpy(src).cuda()
    P, L, S = trw.walk(G, table, p, d_src)      # persistent, default tuning (as timed by bench.py)
    torch.cuda.synchronize()
    return P, L, S


@pytest.mark.timeout(900)
def test_ppr_rmat22_every_query():
    wl = synth.WORKLOADS["ppr-rmat22"]
    g = synth.make_graph(wl)
    src = synth.make_sources(wl, g)
    log(f"  ppr-rmat22: n={g.n} m={g.m} nq={len(src)}")
    G = trw.Graph(g.row_ptr, g.col, g.weight, symmetric=wl.symmetric)
    assert G.validate() == 0
    alias = G.table("alias")
    p = _params(wl, "alias")
    P, L, S = _walk_full(G, alias, p, src)
    Lh, Sh = L.cpu().numpy(), S.cpu().numpy()
    _check_rules(wl, Lh, Sh)
    thr, al = oracle.alias_build(g.row_ptr, g.weight)
    op = _oracle_params(p)
    group = 2_000_000
    exp_counts = np.zeros((len(src) // group, g.n), np.uint32)
    for lo in range(0, len(src), group):
        hi = min(len(src), lo + group)
        ref = _oracle_range(g, op, src, lo, hi, thr=thr, alias=al)
        _compare(P[lo:hi].cpu().numpy(), Lh[lo:hi], Sh[lo:hi], ref, wl.max_len, f"ppr-rmat22 queries {lo}..{hi}")
        log(f"  ppr-rmat22 queries {lo}..{hi} identical")
        # the oracle's end counts of the same queries (one group per range)
        oracle.end_counts(g.n, ref.paths, ref.lengths, ref.status, counts=exp_counts[lo // group])
        del ref
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
    del counts, L2, S2, thr, al
    alias.close()
    # REJ on the same batch: every query
    rej = G.table("rej")
    pr = _params(wl, "rej")
    P, L, S = _walk_full(G, rej, pr, src)
    _check_rules(wl, L.cpu().numpy(), S.cpu().numpy())
    _every_query("ppr-rmat22 REJ", g, src, [(P, L, S)], _oracle_params(pr), wl.max_len,
                 weight=g.weight, pmax=oracle.rej_build(g.row_ptr, g.weight))
    G.close()


@pytest.mark.timeout(900)
def test_node2vec_rmat24_every_query():
    wl = synth.WORKLOADS["node2vec-rmat24"]
    g = synth.make_graph(wl)
    src = synth.make_sources(wl, g)
    log(f"  node2vec-rmat24: n={g.n} m={g.m} nq={len(src)}")
    G = trw.Graph(g.row_ptr, g.col, symmetric=wl.symmetric)
    assert G.validate() == 0
    eidx = G.edge_index()
    p = _params(wl, "orej")
    P, L, S = _walk_full(G, eidx, p, src)
    Lh, Sh = L.cpu().numpy(), S.cpu().numpy()
    _check_rules(wl, Lh, Sh)
    _check_hops(g, P[:300].cpu().numpy(), Lh[:300].view(np.uint32))
    _every_query("node2vec-rmat24", g, src, [(P, L, S)], _oracle_params(p), wl.max_len)
    G.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("sampler", ["its", "rej"])
def test_ppr_rmat22_from_disk_every_query(tmp_path, sampler):
    """The PPR batch with ITS and with REJ walked from a CSR file in 17 partitions, 8
    resident (tables built per partition over its vertex range, partitions evicted and
    reloaded): every query equals the in-memory walk, itself compared with the oracle on
    every query above."""
    wl = synth.WORKLOADS["ppr-rmat22"]
    g = synth.make_graph(wl)
    src = synth.make_sources(wl, g)
    path = str(tmp_path / "ppr22.csr")
    trw.write_disk_graph(path, g.row_ptr.astype(np.int64), g.col, g.weight)
    G = trw.Graph(g.row_ptr, g.col, g.weight)
    p = _params(wl, sampler)
    P, L, S = _walk_full(G, G.table(sampler), p, src)
    D = trw.DiskGraph(path, g.m // 16)
    log(f"  ppr-rmat22 {sampler} from disk: {D.parts} partitions, 8 resident, nq={len(src)}")
    t0 = time.time()
    Pd, Ld, Sd, st = D.walk(p, torch.from_numpy(src).cuda(), slots=8)
    torch.cuda.synchronize()
    log(f"  {time.time() - t0:.2f} s, {st['runs']} rounds, {st['loads']} loads")
    assert torch.equal(Ld, L) and torch.equal(Sd, S)
    cols = torch.arange(wl.max_len + 1, device=P.device)[None, :]
    for a in range(0, len(src), CHUNK):
        b = min(len(src), a + CHUNK)
        keep = cols <= L[a:b, None]
        assert torch.equal(torch.where(keep, Pd[a:b], 0), torch.where(keep, P[a:b, :wl.max_len + 1], 0)), a
    log("  every query identical to the in-memory walk")
    D.close()
    G.close()


@pytest.mark.timeout(900)
def test_node2vec_rmat24_from_disk_every_query(tmp_path):
    """The Node2Vec batch walked from a CSR file in 8 partitions, 4 resident (queries wait
    under pairs of partitions and partitions are evicted and reloaded): every query equals
    the in-memory walk, itself compared with the oracle on every query above."""
    wl = synth.WORKLOADS["node2vec-rmat24"]
    g = synth.make_graph(wl)
    src = synth.make_sources(wl, g)
    path = str(tmp_path / "n2v24.csr")
    trw.write_disk_graph(path, g.row_ptr.astype(np.int64), g.col)
    G = trw.Graph(g.row_ptr, g.col, symmetric=wl.symmetric)
    p = _params(wl, "orej")
    P, L, S = _walk_full(G, G.edge_index(), p, src)
    D = trw.DiskGraph(path, g.m // 8 + 1)
    log(f"  node2vec-rmat24 from disk: {D.parts} partitions, 4 resident, nq={len(src)}")
    t0 = time.time()
    Pd, Ld, Sd, st = D.walk(p, torch.from_numpy(src).cuda(), slots=4)
    torch.cuda.synchronize()
    log(f"  {time.time() - t0:.1f} s, {st['runs']} rounds, {st['loads']} loads, {st['bytes_read'] / 1e9:.1f} GB read")
    assert torch.equal(Ld, L) and torch.equal(Sd, S)
    cols = torch.arange(wl.max_len + 1, device=P.device)[None, :]
    for a in range(0, len(src), CHUNK):
        b = min(len(src), a + CHUNK)
        keep = cols <= L[a:b, None]
        assert torch.equal(torch.where(keep, Pd[a:b], 0), torch.where(keep, P[a:b, :wl.max_len + 1], 0)), a
    log("  every query identical to the in-memory walk")
    D.close()
    G.close()


@pytest.mark.timeout(900)
def test_metapath_rmat24_every_query():
    """With the label index and by row scans: both equal the oracle on every query."""
    wl = synth.WORKLOADS["metapath-rmat24"]
    g = synth.make_graph(wl)
    src = synth.make_sources(wl, g)
    log(f"  metapath-rmat24: n={g.n} m={g.m} nq={len(src)}")
    G = trw.Graph(g.row_ptr, g.col, None, g.label, symmetric=wl.symmetric)
    assert G.validate() == 0
    index = G.label_index(wl.labels)
    p = _params(wl, "its")
    P, L, S = _walk_full(G, index, p, src)
    _check_rules(wl, L.cpu().numpy(), S.cpu().numpy())
    P2, L2, S2 = _walk_full(G, None, p, src)             # row scans
    _every_query("metapath-rmat24, label index and row scans", g, src, [(P, L, S), (P2, L2, S2)],
                 _oracle_params(p), wl.max_len, label=g.label)
    G.close()


@pytest.mark.timeout(900)
def test_served_rmat26_saturated_replay_every_query():
    """The bench's first replay of the served mix (2000 requests, all submitted at once) through
    the server in the bench's configuration; every query of every request against the oracle."""
    import ctypes
    from paper_2107_11983_amd import _abi
    wl = synth.WORKLOADS["served-rmat26"]
    g = synth.make_graph(wl)
    log(f"  served-rmat26: n={g.n} m={g.m}")
    G = trw.Graph(g.row_ptr, g.col, g.weight, symmetric=True)
    assert G.validate() == 0
    alias = G.table("alias")
    eidx = G.edge_index()
    R = 2000
    sizes, kinds, offs, src = synth.served_requests(wl, R, g.n)
    algo_p = [trw.make_params("deepwalk", "alias", 80, wl.walk_seed),
              trw.make_params("ppr", "alias", 256, wl.walk_seed, stop_q32=trw.stop_threshold(wl.stop_prob)),
              trw.make_params("node2vec", "orej", 80, wl.walk_seed, n2v_thr_q16=trw.n2v_thresholds(*wl.n2v_pq))]
    strides = np.array([88, 264, 88])
    poff = np.concatenate([[0], np.cumsum(sizes * strides[kinds])])
    d_src = torch.from_numpy(src).cuda()
    d_paths = torch.full((int(poff[-1]),), -7, dtype=torch.int32, device="cuda")
    d_len = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
    d_st = torch.empty(int(offs[-1]), dtype=torch.uint8, device="cuda")
    reqs = (_abi.trw_request * R)()
    for i in range(R):
        r = reqs[i]
        r.params = algo_p[kinds[i]]
        r.nq = int(sizes[i])
        r.sources = ctypes.c_void_p(d_src.data_ptr() + 4 * int(offs[i]))
        r.qid_base = i << 32
        r.paths = ctypes.c_void_p(d_paths.data_ptr() + 4 * int(poff[i]))
        r.path_stride = int(strides[kinds[i]])
        r.lengths = ctypes.c_void_p(d_len.data_ptr() + 4 * int(offs[i]))
        r.status = ctypes.c_void_p(d_st.data_ptr() + int(offs[i]))
    torch.cuda.synchronize()
    slots = torch.cuda.get_device_properties(0).multi_processor_count * 4096
    srv = trw.Server(G, alias, eidx, pool_bytes=8 << 30, max_slots=slots, max_requests=4096, steps_per_tick=64)
    comp = (_abi.trw_completion * R)()
    arr = (ctypes.c_uint64 * R)()
    t0 = time.time()
    rc = _abi.trw_probe_serve_replay(srv.handle, R, reqs, arr, comp, 600_000)
    assert rc == 0, f"replay failed: {rc} {_abi.trw_last_error()}"
    assert all(comp[i].status == 0 for i in range(R))
    log(f"  served-rmat26: {R} requests ({int(offs[-1])} queries) served in {time.time() - t0:.2f}s, "
        f"{srv.stats()['ticks']} ticks")
    srv.close()
    paths = d_paths.cpu().numpy()
    lengths = d_len.cpu().numpy().view(np.uint32)
    status = d_st.cpu().numpy()
    thr, al = oracle.alias_build(g.row_ptr, g.weight)
    ops = [_oracle_params(p) for p in algo_p]

    def run(i):
        kw = dict(thr=thr, alias=al) if kinds[i] < 2 else {}
        return oracle.walk(g.row_ptr, g.col, ops[kinds[i]], src[offs[i]:offs[i + 1]], qid_base=i << 32, **kw)
    t0 = time.time()
    moves = 0
    with concurrent.futures.ThreadPoolExecutor(max_workers=WORKERS) as ex:
        for i, ref in enumerate(ex.map(run, range(R))):
            nq, stride, ml = int(sizes[i]), int(strides[kinds[i]]), int(algo_p[kinds[i]].max_len)
            P = paths[poff[i]:poff[i + 1]].reshape(nq, stride)
            _compare(P, lengths[offs[i]:offs[i + 1]], status[offs[i]:offs[i + 1]], ref, ml, f"served request {i}")
            moves += int(ref.lengths.sum())
    log(f"  served-rmat26: every query of {R} requests identical ({int(offs[-1])} queries, {moves} moves, "
        f"oracle on {WORKERS} threads {time.time() - t0:.1f}s)")
    G.close()
