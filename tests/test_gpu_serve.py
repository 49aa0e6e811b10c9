"""The continuous-batching server through the C ABI (trw_server_*).

Each request's result must be bit-identical to the same request walked alone,
in any mix of concurrent requests, through trw_walk, and by the oracle;
cancellation and memory admission must leave other requests untouched.
"""
import sys
import time

import numpy as np
import pytest
import torch

import oracle
import synth

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
    g = synth.rmat(12, 16, True, 0x5E4E)
    synth.attach_attrs(g, 0x5E4E ^ 1, weights=True)
    G = trw.Graph(g.row_ptr, g.col, g.weight, symmetric=True)
    assert G.validate() == 0
    alias = G.table("alias")
    adj = G.adjacency_index()
    eidx = G.edge_index()
    thr, al = oracle.alias_build(g.row_ptr, g.weight)
    torch.cuda.synchronize()
    return dict(g=g, G=G, alias=alias, adj=adj, eidx=eidx, orc_alias=(thr, al))


SERVED = [("deepwalk", "alias", 80), ("ppr", "alias", 256), ("node2vec", "orej", 80),
          ("deepwalk", "naive", 40), ("ppr", "naive", 64)]


def params(algo, sampler, max_len, seed):
    kw = {}
    if algo == "ppr":
        kw["stop_q32"] = trw.stop_threshold(0.2)
    if algo == "node2vec":
        kw["n2v_thr_q16"] = trw.n2v_thresholds(2.0, 0.5)
    return trw.make_params(algo, sampler, max_len, seed, **kw)


def wait_all(server, ids, timeout_s=60.0):
    got = {}
    t0 = time.time()
    while len(got) < len(ids):
        assert time.time() - t0 < timeout_s, f"requests did not complete: {set(ids) - set(got)}"
        for c in server.poll(256, timeout_ms=50):
            got[c["request_id"]] = c
    return got


def to_np(c):
    P = c["paths"].cpu().numpy() if isinstance(c["paths"], torch.Tensor) else c["paths"]
    L = c["lengths"].cpu().numpy().view(np.uint32) if isinstance(c["lengths"], torch.Tensor) else c["lengths"]
    S = c["status_codes"].cpu().numpy() if isinstance(c["status_codes"], torch.Tensor) else c["status_codes"]
    return P, L, S


def same(a, b, max_len):
    Pa, La, Sa = a
    Pb, Lb, Sb = b
    assert np.array_equal(La, Lb) and np.array_equal(Sa, Sb)
    mask = np.arange(max_len + 1)[None, :] <= La[:, None]
    assert np.array_equal(Pa[:, :max_len + 1][mask], Pb[:, :max_len + 1][mask])


def make_server(env, index="adj", **kw):
    cfg = dict(pool_bytes=256 << 20, max_slots=256 * 64, steps_per_tick=16)
    cfg.update(kw)
    return trw.Server(env["G"], env["alias"], env[index], **cfg)


@pytest.mark.parametrize("index", ["adj", "eidx"])
def test_served_equals_walk_and_oracle(env, index):
    g = env["g"]
    srv = make_server(env, index=index)
    src = synth.sources(777, g.n, 31)
    for algo, sampler, max_len in SERVED:
        log(f"  served {algo}/{sampler}")
        p = params(algo, sampler, max_len, 99)
        rid = srv.submit(p, src, qid_base=5000)
        c = wait_all(srv, [rid])[rid]
        assert c["status"] == 0
        got = to_np(c)
        table = env["alias"] if sampler == "alias" else None
        P, L, S = trw.walk(env["G"], table, p, torch.from_numpy(src).cuda(), qid_base=5000)
        torch.cuda.synchronize()
        same(got, (P.cpu().numpy(), L.cpu().numpy().view(np.uint32), S.cpu().numpy()), max_len)
        kw = {}
        if sampler == "alias":
            kw = dict(thr=env["orc_alias"][0], alias=env["orc_alias"][1])
        op = oracle.WalkParams(oracle.ALGOS[algo], oracle.SAMPLERS[sampler], max_len, 99,
                               stop_q32=p.stop_q32, n2v_thr_q16=tuple(p.n2v_thr_q16))
        ref = oracle.walk(g.row_ptr, g.col, op, src, qid_base=5000, **kw)
        same(got, (ref.paths, ref.lengths, ref.status), max_len)
    srv.close()


def _mix(g, n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        algo, sampler, max_len = SERVED[int(rng.integers(0, len(SERVED)))]
        nq = int(rng.integers(1, 400))
        reqs.append((algo, sampler, max_len, synth.sources(nq, g.n, seed * 1000 + i), 1000 * i, 7 + i))
    return reqs


@pytest.mark.parametrize("use_graph,pipelined", [(True, False), (False, False), (True, True)])
def test_same_alone_and_in_mix(env, use_graph, pipelined):
    g = env["g"]
    reqs = _mix(g, 30, 5)
    srv = make_server(env, use_hipgraph=use_graph, pipelined=pipelined)
    alone = []
    for algo, sampler, max_len, src, qb, seed in reqs:
        rid = srv.submit(params(algo, sampler, max_len, seed), src, qid_base=qb)
        alone.append(to_np(wait_all(srv, [rid])[rid]))
    ids = [srv.submit(params(a, s, m, seed), src, qid_base=qb) for a, s, m, src, qb, seed in reqs]
    got = wait_all(srv, ids)
    st = srv.stats()
    log(f"  stats {st}")
    for (algo, sampler, max_len, *_), rid, ref in zip(reqs, ids, alone):
        assert got[rid]["status"] == 0
        same(to_np(got[rid]), ref, max_len)
    assert st["completed"] == 60 and st["active"] == 0
    srv.close()


@pytest.mark.parametrize("pipelined", [False, True])
def test_cancel_leaves_others_intact(env, pipelined):
    g = env["g"]
    srv = make_server(env, pipelined=pipelined)
    small = _mix(g, 6, 9)
    alone = []
    for algo, sampler, max_len, src, qb, seed in small:
        rid = srv.submit(params(algo, sampler, max_len, seed), src, qid_base=qb)
        alone.append(to_np(wait_all(srv, [rid])[rid]))
    # large enough (48 M moves) that it is still running when the cancel arrives
    big = srv.submit(params("node2vec", "orej", 80, 3), synth.sources(600000, g.n, 4), qid_base=10 ** 9)
    ids = [srv.submit(params(a, s, m, seed), src, qid_base=qb) for a, s, m, src, qb, seed in small]
    moves0 = srv.stats()["moves"]
    t0 = time.time()
    while srv.stats()["moves"] == moves0:
        assert time.time() - t0 < 10, "the server made no progress"
        time.sleep(0.0002)
    srv.cancel(big)
    got = wait_all(srv, ids + [big])
    assert got[big]["status"] == trw.TRW_E_CANCELLED
    for (algo, sampler, max_len, *_), rid, ref in zip(small, ids, alone):
        assert got[rid]["status"] == 0
        same(to_np(got[rid]), ref, max_len)
    srv.close()


def test_memory_admission(env):
    """Requests with host buffers are staged in the pool: one that can never fit
    is refused, and ones that fit only one at a time are admitted in turn."""
    g = env["g"]
    p = params("deepwalk", "alias", 80, 1)
    srv = make_server(env, pool_bytes=4 << 20)
    with pytest.raises(trw.TrwError) as ei:
        srv.submit(p, synth.sources(20000, g.n, 1), host=True)   # 20000 * (88 * 4 + 9) bytes > 4 MiB
    assert ei.value.status == trw.TRW_E_NOMEM_BUDGET
    # each fits alone but no two fit together: admitted one after another
    reqs = [synth.sources(7000, g.n, 10 + i) for i in range(4)]
    ids = [srv.submit(p, s, qid_base=i << 20, host=True) for i, s in enumerate(reqs)]
    got = wait_all(srv, ids)
    for i, (s, rid) in enumerate(zip(reqs, ids)):
        P, L, S = trw.walk(env["G"], env["alias"], p, torch.from_numpy(s).cuda(), qid_base=i << 20)
        torch.cuda.synchronize()
        same(to_np(got[rid]), (P.cpu().numpy(), L.cpu().numpy().view(np.uint32), S.cpu().numpy()), 80)
        assert got[rid]["t_admit_ns"] >= got[rid]["t_submit_ns"]
    admits = sorted(got[r]["t_admit_ns"] for r in ids)
    dones = sorted(got[r]["t_done_ns"] for r in ids)
    assert all(admits[i + 1] >= dones[i] - 10 ** 9 for i in range(3))
    srv.close()


def test_device_buffers_in_place(env):
    """Requests with device buffers take no pool space: written in place, they
    run together even when their outputs together are far larger than the pool,
    and give the same results as the batch walker."""
    g = env["g"]
    srv = make_server(env, pool_bytes=4 << 20)
    kinds = [("deepwalk", "alias", 80), ("ppr", "alias", 256), ("node2vec", "orej", 80)]
    reqs = [(kinds[i % 3], synth.sources(20000, g.n, 40 + i)) for i in range(6)]
    ids = [srv.submit(params(a, s, m, 5 + i), src, qid_base=i << 24)
           for i, ((a, s, m), src) in enumerate(reqs)]
    assert srv.stats()["pool_bytes_used"] == 0
    got = wait_all(srv, ids)
    for i, (((a, s, m), src), rid) in enumerate(zip(reqs, ids)):
        assert got[rid]["status"] == 0
        table = env["alias"] if s == "alias" else env["eidx"]
        P, L, S = trw.walk(env["G"], table, params(a, s, m, 5 + i), torch.from_numpy(src).cuda(), qid_base=i << 24)
        torch.cuda.synchronize()
        same(to_np(got[rid]), (P.cpu().numpy(), L.cpu().numpy().view(np.uint32), S.cpu().numpy()), m)
    srv.close()


@pytest.mark.parametrize("stride", [81, 83, 97])
def test_in_place_rows_of_any_stride(env, stride):
    """Device rows written in place at a stride that is not a multiple of 4 entries (rows
    start at every 4-byte alignment, so the writer mixes single entries and 16-byte blocks):
    the entries up to each path's end equal the batch walker's."""
    g = env["g"]
    srv = make_server(env)
    kinds = [("deepwalk", "alias", 80), ("node2vec", "orej", 80), ("ppr", "alias", 64)]
    ids, reqs = [], []
    for i, (a, s, m) in enumerate(kinds):
        src = synth.sources(3001, g.n, 70 + i)
        p = params(a, s, m, 9 + i)
        rid = srv.submit(p, src, qid_base=i << 20, stride=stride)
        ids.append(rid)
        reqs.append((a, s, m, src, p, rid))
    got = wait_all(srv, ids)
    for i, (a, s, m, src, p, rid) in enumerate(reqs):
        P, L, S = to_np(got[rid])
        assert P.shape[1] == stride
        table = env["alias"] if s == "alias" else env["eidx"]
        Pr, Lr, Sr = trw.walk(env["G"], table, p, torch.from_numpy(src).cuda(), qid_base=i << 20)
        torch.cuda.synchronize()
        same((P, L, S), (Pr.cpu().numpy(), Lr.cpu().numpy().view(np.uint32), Sr.cpu().numpy()), m)
    srv.close()


def test_extreme_requests(env):
    """One query, max_len 1, and requests larger than every other in flight, of each kind,
    submitted together with bad sources at both ends: each equals the batch walker and the
    oracle's termination rules."""
    g = env["g"]
    srv = make_server(env, steps_per_tick=7)      # a tick length that divides no walk evenly
    cases = []
    for i, (a, s, m) in enumerate([("deepwalk", "alias", 1), ("ppr", "alias", 1), ("node2vec", "orej", 1),
                                   ("deepwalk", "alias", 80), ("ppr", "alias", 256), ("node2vec", "orej", 80)]):
        n = 1 if i < 3 else 70001
        src = synth.sources(n, g.n, 90 + i)
        if n > 2:
            src[0], src[-1] = -1, g.n                 # bad sources at both ends of the request
        cases.append((a, s, m, src, params(a, s, m, 31 + i), i << 24))
    ids = [srv.submit(p, src, qid_base=qb) for a, s, m, src, p, qb in cases]
    got = wait_all(srv, ids)
    for (a, s, m, src, p, qb), rid in zip(cases, ids):
        assert got[rid]["status"] == 0
        table = env["alias"] if s == "alias" else env["eidx"]
        Pr, Lr, Sr = trw.walk(env["G"], table, p, torch.from_numpy(src).cuda(), qid_base=qb)
        torch.cuda.synchronize()
        P, L, S = to_np(got[rid])
        Sr = Sr.cpu().numpy()
        assert np.array_equal(L, Lr.cpu().numpy().view(np.uint32)) and np.array_equal(S, Sr)
        ok = Sr != oracle.ST_BAD_SOURCE
        mask = (np.arange(m + 1)[None, :] <= L[:, None]) & ok[:, None]
        assert np.array_equal(P[:, :m + 1][mask], Pr.cpu().numpy()[:, :m + 1][mask])
        if len(src) > 2:
            assert S[0] == oracle.ST_BAD_SOURCE and S[-1] == oracle.ST_BAD_SOURCE and L[0] == 0
    srv.close()


def test_host_buffers_and_bad_sources(env):
    g = env["g"]
    srv = make_server(env)
    src = np.array([0, -5, g.n, 17, 4095], np.int32)
    p = params("ppr", "alias", 256, 11)
    rid = srv.submit(p, src, host=True)
    c = wait_all(srv, [rid])[rid]
    P, L, S = c["paths"], c["lengths"], c["status_codes"]
    assert list(S[[1, 2]]) == [trw.TRW_ST_BAD_SOURCE] * 2 and list(L[[1, 2]]) == [0, 0]
    Pd, Ld, Sd = trw.walk(env["G"], env["alias"], p, torch.from_numpy(src).cuda())
    torch.cuda.synchronize()
    Ld, Sd = Ld.cpu().numpy().view(np.uint32), Sd.cpu().numpy()
    assert np.array_equal(L, Ld) and np.array_equal(S, Sd)
    for i in (0, 3, 4):
        assert np.array_equal(P[i, :L[i] + 1], Pd.cpu().numpy()[i, :L[i] + 1])
    srv.close()


def test_rejects_unsupported(env):
    srv = make_server(env)
    with pytest.raises(trw.TrwError) as ei:
        srv.submit(trw.make_params("metapath", "its", 10, 1, schema=(1,)), np.zeros(4, np.int32))
    assert ei.value.status == trw._abi.TRW_E_UNSUPPORTED
    srv.close()
    noalias = trw.Server(env["G"], None, None, pool_bytes=1 << 20, max_slots=256)
    with pytest.raises(trw.TrwError):
        noalias.submit(params("deepwalk", "alias", 5, 1), np.zeros(4, np.int32))
    noalias.close()


def test_small_ring_admits_more_than_it_holds(env):
    """A ring of 16 chunks (requests of at most 511 queries) and 40 requests holding
    about 200 chunks in all, submitted at once: admission waits for ring entries the
    device has read, so no published chunk is overwritten and every request's result
    equals the same walk through trw_walk."""
    g = env["g"]
    srv = make_server(env, ring_chunks=16)
    with pytest.raises(trw.TrwError) as ei:
        srv.submit(params("deepwalk", "alias", 80, 1), synth.sources(512, g.n, 1))
    assert ei.value.status == trw.TRW_E_INVALID
    rng = np.random.default_rng(17)
    reqs = []
    for i in range(40):
        algo, sampler, max_len = SERVED[i % len(SERVED)]
        nq = int(rng.integers(64, 512))
        reqs.append((algo, sampler, max_len, synth.sources(nq, g.n, 900 + i), (i + 1) << 24, 40 + i))
    assert sum(-(-len(r[3]) // 64) for r in reqs) > 10 * 16
    ids = [srv.submit(params(a, s, m, seed), src, qid_base=qb) for a, s, m, src, qb, seed in reqs]
    got = wait_all(srv, ids)
    for (algo, sampler, max_len, src, qb, seed), rid in zip(reqs, ids):
        assert got[rid]["status"] == 0
        p = params(algo, sampler, max_len, seed)
        table = env["alias"] if sampler == "alias" else None
        P, L, S = trw.walk(env["G"], table, p, torch.from_numpy(src).cuda(), qid_base=qb)
        torch.cuda.synchronize()
        same(to_np(got[rid]), (P.cpu().numpy(), L.cpu().numpy().view(np.uint32), S.cpu().numpy()), max_len)
    assert srv.stats()["completed"] == 40
    srv.close()
