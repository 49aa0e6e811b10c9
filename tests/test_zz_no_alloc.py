"""trw_walk_noalloc through the C ABI: the walk with the library's own device
workspace gives the same bits as trw_walk with a caller workspace, on two
calls in a row (the second smaller, so the array still holds the first call's
contents), for both schedules and for walks with and without tables."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

trw = None


@pytest.fixture(scope="module")
def env():
    global trw
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2107_11983_amd as mod
    trw = mod
    torch.cuda.set_device(0)
    g = synth.rmat(14, 16, True, 0x0A110C)
    synth.attach_attrs(g, 0x0A110C ^ 3, weights=True)
    G = trw.Graph(g.row_ptr, g.col, g.weight, symmetric=True)
    assert G.validate() == 0
    tables = {"alias": G.table("alias"), "eidx": G.edge_index()}
    torch.cuda.synchronize()
    return dict(g=g, G=G, tables=tables)


CASES = [("ppr", "alias", 256, "alias"), ("deepwalk", "naive", 80, None), ("node2vec", "orej", 40, "eidx")]


def _params(algo, sampler, max_len, seed):
    kw = {}
    if algo == "ppr":
        kw["stop_q32"] = trw.stop_threshold(0.2)
    if algo == "node2vec":
        kw["n2v_thr_q16"] = trw.n2v_thresholds(2.0, 0.5)
    return trw.make_params(algo, sampler, max_len, seed, **kw)


def _same(a, b, max_len):
    Pa, La, Sa = (x.cpu().numpy() for x in a)
    Pb, Lb, Sb = (x.cpu().numpy() for x in b)
    assert np.array_equal(La, Lb) and np.array_equal(Sa, Sb)
    mask = np.arange(max_len + 1)[None, :] <= La.view(np.uint32)[:, None]
    assert np.array_equal(Pa[:, :max_len + 1][mask], Pb[:, :max_len + 1][mask])


@pytest.mark.parametrize("mode", ["persistent", "per_step"])
@pytest.mark.parametrize("algo,sampler,max_len,table", CASES)
def test_noalloc_equals_walk_two_calls(env, algo, sampler, max_len, table, mode):
    g, G = env["g"], env["G"]
    tab = env["tables"][table] if table else None
    p = _params(algo, sampler, max_len, 0xA110C)
    for call, (nq, seed, qb) in enumerate([(60000, 1, 0), (7001, 2, 1 << 33)]):
        src = torch.from_numpy(synth.sources(nq, g.n, seed)).cuda()
        ref = trw.walk(G, tab, p, src, qid_base=qb, mode=mode)
        stride = (max_len + 1 + 15) // 16 * 16
        out = (torch.full((nq, stride), -3, dtype=torch.int32, device="cuda"),
               torch.empty(nq, dtype=torch.int32, device="cuda"), torch.empty(nq, dtype=torch.uint8, device="cuda"))
        got = trw.walk_noalloc(G, tab, p, src, *out, qid_base=qb, mode=mode)
        torch.cuda.synchronize()
        _same(got, ref, max_len)
        print(f"  {algo}/{sampler} {mode} call {call}: {nq} queries identical", flush=True)
    # the second call's queries against the oracle too
    kw = {}
    if sampler == "alias":
        thr, al = oracle.alias_build(g.row_ptr, g.weight)
        kw = dict(thr=thr, alias=al)
    op = oracle.WalkParams(oracle.ALGOS[algo], oracle.SAMPLERS[sampler], max_len, 0xA110C, stop_q32=p.stop_q32,
                           n2v_thr_q16=tuple(p.n2v_thr_q16))
    r = oracle.walk(g.row_ptr, g.col, op, src.cpu().numpy(), qid_base=1 << 33, **kw)
    L = got[1].cpu().numpy().view(np.uint32)
    assert np.array_equal(L, r.lengths) and np.array_equal(got[2].cpu().numpy(), r.status)


def test_noalloc_rejects_beyond_its_scratch(env):
    g, G = env["g"], env["G"]
    p = _params("deepwalk", "naive", 80, 5)
    nq = 300000                                   # per step: 2 x 16 B per query > 8 MiB
    src = torch.zeros(nq, dtype=torch.int32, device="cuda")
    out = (torch.empty((nq, 96), dtype=torch.int32, device="cuda"), torch.empty(nq, dtype=torch.int32, device="cuda"),
           torch.empty(nq, dtype=torch.uint8, device="cuda"))
    with pytest.raises(trw.TrwError) as ei:
        trw.walk_noalloc(G, None, p, src, *out, mode="per_step")
    assert ei.value.status == trw.TRW_E_INVALID
