"""PPR estimate on the GPU (through the C ABI) against the oracle.

End counts: the oracle walks and counts on its own; the GPU walks and counts
on its own; the counts must be equal (they are integers).  Hand-built outputs
with bad sources, lengths past the row and ends outside the graph check the
skip rules.  Top-k: equal to the oracle's (a full sort cut at k) on counts
with many ties, large values, all-equal rows, k = 1, k = n and k = 4096.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

trw = None


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


@pytest.fixture(scope="module")
def rmat_dir():
    g = synth.rmat(12, 16, False, 0xE2D)
    synth.attach_attrs(g, 0xE2D ^ 3, weights=True)
    return g


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("sampler", ["alias", "rej"])
@pytest.mark.parametrize("group", [0, 1000, 7])
def test_end_counts_match_oracle(rmat_dir, sampler, group):
    g = rmat_dir
    G = trw.Graph(g.row_ptr, g.col, g.weight)
    table = G.table(sampler)
    n = g.n
    # single-source groups (the paper's PPR: many queries from one source) and uniform sources
    src = np.concatenate([np.repeat(np.array([3, 77, 1000], np.int32), 2000),
                          synth.sources(5003, n, 41), np.array([-1, n], np.int32)])
    stop = oracle.stop_q32(0.2)
    log(f"  end counts {sampler} group={group} nq={len(src)}")
    p = trw.make_params("ppr", sampler, 256, 123, stop_q32=stop)
    P, L, S = trw.walk(G, table, p, torch.from_numpy(src).cuda())
    counts, skipped = trw.ppr_end_counts(G, P, L, S, group=group)
    torch.cuda.synchronize()
    kw = (dict(zip(("thr", "alias"), oracle.alias_build(g.row_ptr, g.weight))) if sampler == "alias"
          else dict(weight=g.weight, pmax=oracle.rej_build(g.row_ptr, g.weight)))
    ref = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.PPR, oracle.SAMPLERS[sampler], 256, 123,
                                                          stop_q32=stop), src, **kw)
    exp, exp_skipped = oracle.end_counts(n, ref.paths, ref.lengths, ref.status, group=group)
    assert exp_skipped == 2
    assert int(skipped.item()) == exp_skipped
    assert np.array_equal(_u32(counts).reshape(exp.shape), exp)
    # the scores are shares of each group's queries
    if group == 0:
        assert int(_u32(counts).sum()) == len(src) - 2
    G.close()


def test_end_counts_skip_rules_and_accumulate():
    g = synth.from_edges(6, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5)])
    G = trw.Graph(g.row_ptr, g.col)
    rng = np.random.default_rng(5)
    nq, stride = 3001, 9
    paths = rng.integers(-3, 9, size=(nq, stride)).astype(np.int32)     # some ends outside [0, 6)
    lengths = rng.integers(0, 11, size=nq).astype(np.uint32)            # some past the row
    status = rng.integers(1, 5, size=nq).astype(np.uint8)               # some bad sources
    dP = torch.from_numpy(paths).cuda()
    dL = torch.from_numpy(lengths.view(np.int32)).cuda()
    dS = torch.from_numpy(status).cuda()
    for group in (0, 1, 64, 3000, 5000):
        counts, skipped = trw.ppr_end_counts(G, dP, dL, dS, group=group)
        counts, skipped = trw.ppr_end_counts(G, dP, dL, dS, group=group, counts=counts, skipped=skipped)
        torch.cuda.synchronize()
        exp, sk = oracle.end_counts(6, paths, lengths, status, group=group)
        exp, sk2 = oracle.end_counts(6, paths, lengths, status, group=group, counts=exp)
        assert int(skipped.item()) == sk + sk2 and sk > 0
        assert np.array_equal(_u32(counts).reshape(exp.shape), exp), group
    # an empty batch is a no-op; a short counts buffer is refused
    counts, skipped = trw.ppr_end_counts(G, dP[:0], dL[:0], dS[:0])
    assert int(counts.sum().item()) == 0
    with pytest.raises(trw.TrwError):
        trw.ppr_end_counts(G, dP, dL, dS, group=1000, counts=torch.zeros((2, 6), dtype=torch.int32, device="cuda"))
    G.close()


def _counts_cases():
    rng = np.random.default_rng(99)
    yield "ties", rng.integers(0, 6, size=100_003).astype(np.uint32)
    yield "geometric", rng.geometric(0.01, size=1 << 22).astype(np.uint32)
    yield "large", (0xFFFFFFFF - rng.integers(0, 50, size=70_001)).astype(np.uint32)
    yield "equal", np.full(5000, 7, np.uint32)
    yield "zeros_one_hot", np.where(np.arange(300_000) == 123_456, 1, 0).astype(np.uint32)
    yield "tiny", np.array([5], np.uint32)
    yield "spread", rng.permutation(200_000).astype(np.uint32)


@pytest.mark.parametrize("name,counts", list(_counts_cases()), ids=[c[0] for c in _counts_cases()])
def test_topk_matches_oracle(name, counts):
    d = torch.from_numpy(counts.view(np.int32)).cuda()
    n = len(counts)
    for k in sorted({1, 7, 100, min(n, 4096), min(n, 4095), n if n <= 4096 else 1}):
        if k > n:
            continue
        ids, vals = trw.topk(d, k)
        torch.cuda.synchronize()
        eid, evals = oracle.topk(counts, k)
        log(f"  topk {name} n={n} k={k}")
        assert np.array_equal(ids.cpu().numpy(), eid), (name, k)
        assert np.array_equal(vals.cpu().numpy().view(np.uint32), evals), (name, k)


def test_topk_rejects_bad_arguments():
    d = torch.zeros(10, dtype=torch.int32, device="cuda")
    with pytest.raises(trw.TrwError):
        trw.topk(d, 11)
    big = torch.zeros(5000, dtype=torch.int32, device="cuda")
    with pytest.raises(trw.TrwError):
        trw.topk(big, 4097)
    ids, vals = trw.topk(d, 0)
    assert ids.numel() == 0 and vals.numel() == 0


@pytest.mark.parametrize("sampler,index", [("alias", None), ("its", None), ("rej", None), ("naive", None),
                                           ("naive", "adj")])
@pytest.mark.parametrize("group,wpl", [(0, 0), (1000, 2), (7, 4), (0, 1)])
def test_ppr_walk_counts_match_oracle(rmat_dir, sampler, index, group, wpl):
    """Counting walks (no paths) give the oracle's end counts, lengths and status."""
    g = rmat_dir
    G = trw.Graph(g.row_ptr, g.col, g.weight)
    table = G.adjacency_index() if index == "adj" else (G.table(sampler) if sampler != "naive" else None)
    n = g.n
    src = np.concatenate([np.repeat(np.array([5, 900], np.int32), 3000), synth.sources(4099, n, 43),
                          np.array([-5, n + 1], np.int32)])
    stop = oracle.stop_q32(0.2)
    p = trw.make_params("ppr", sampler, 256, 321, stop_q32=stop)
    tu = trw.make_tuning(walkers_per_lane=wpl) if wpl else None
    log(f"  counting walk {sampler}/{index} group={group} wpl={wpl} nq={len(src)}")
    counts, L, S = trw.ppr_walk_counts(G, table, p, torch.from_numpy(src).cuda(), group=group, qid_base=11,
                                       tuning=tu)
    torch.cuda.synchronize()
    kw = {}
    if sampler == "alias":
        kw = dict(zip(("thr", "alias"), oracle.alias_build(g.row_ptr, g.weight)))
    elif sampler == "its":
        kw = dict(prefix=oracle.its_build(g.row_ptr, g.weight))
    elif sampler == "rej":
        kw = dict(weight=g.weight, pmax=oracle.rej_build(g.row_ptr, g.weight))
    ref = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.PPR, oracle.SAMPLERS[sampler], 256, 321,
                                                          stop_q32=stop), src, qid_base=11, **kw)
    exp, skipped = oracle.end_counts(n, ref.paths, ref.lengths, ref.status, group=group)
    assert skipped == 2
    assert np.array_equal(L.cpu().numpy().view(np.uint32), ref.lengths)
    assert np.array_equal(S.cpu().numpy(), ref.status)
    assert np.array_equal(_u32(counts).reshape(exp.shape), exp)
    G.close()


@pytest.mark.parametrize("sampler", ["alias", "its"])
def test_ppr_walk_counts_without_outputs(rmat_dir, sampler):
    """Without lengths and status the counting walk stores only the counts, the same counts."""
    g = rmat_dir
    G = trw.Graph(g.row_ptr, g.col, g.weight)
    table = G.table(sampler)
    src = np.concatenate([synth.sources(9001, g.n, 47), np.array([-3], np.int32)])
    p = trw.make_params("ppr", sampler, 256, 99, stop_q32=oracle.stop_q32(0.2))
    d_src = torch.from_numpy(src).cuda()
    a, L, S = trw.ppr_walk_counts(G, table, p, d_src, group=1000)
    b, L2, S2 = trw.ppr_walk_counts(G, table, p, d_src, group=1000, outputs=False)
    torch.cuda.synchronize()
    assert L2 is None and S2 is None
    assert torch.equal(a, b) and int(b.sum().item()) == len(src) - 1
    G.close()


def test_ppr_walk_counts_rejects_bad_arguments(rmat_dir):
    g = rmat_dir
    G = trw.Graph(g.row_ptr, g.col, g.weight)
    src = torch.zeros(10, dtype=torch.int32, device="cuda")
    with pytest.raises(trw.TrwError):           # not a PPR walk
        trw.ppr_walk_counts(G, None, trw.make_params("deepwalk", "naive", 10, 1), src)
    with pytest.raises(trw.TrwError):           # counts too short for 4 groups
        trw.ppr_walk_counts(G, None, trw.make_params("ppr", "naive", 10, 1), src, group=3,
                            counts=torch.zeros((3, g.n), dtype=torch.int32, device="cuda"))
    with pytest.raises(trw.TrwError):           # ALIAS without its table
        trw.ppr_walk_counts(G, None, trw.make_params("ppr", "alias", 10, 1), src)
    G.close()
