"""The largest graph the ABI takes: m = 2^31 - 1 directed edges.

Row offsets then run up to the int32 limit, and ALIAS entries (32 bytes per
slot, 69 GB) sit at byte offsets near 2^36, so any 32-bit slip in the walk's
or the build's index arithmetic shows.  The graph: n = 2^21 vertices, row v
holds every vertex congruent to v + 1 modulo 2048 (1024 destinations, sorted
by construction, no self-loops), the last row one short; weights uniform in
[1, 255].  Checked against the oracle: the ALIAS entries of rows at both ends
of the table, PPR with ALIAS and DeepWalk with NAIVE from sources that
include the last rows.  Needs about 90 GB of device memory and 35 GB of host
memory; skipped on a smaller device.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

N = 1 << 21
DEG = 1024
M = N * DEG - 1                     # 2^31 - 1


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def big():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.empty_cache()                        # what earlier tests left in torch's cache
    free, _ = torch.cuda.mem_get_info()
    if free < 110 * (1 << 30):
        pytest.skip(f"needs ~110 GB of free device memory, {free >> 30} GB free")
    import paper_2107_11983_amd as trw
    log("  max size: building the 2^31 - 1 edge graph on the host")
    stride = N // DEG
    r = ((np.arange(N, dtype=np.int32) + 1) % stride).astype(np.int32)
    col = (r[:, None] + (stride * np.arange(DEG, dtype=np.int32))[None, :]).ravel()[:M]
    row_ptr = np.minimum(np.arange(N + 1, dtype=np.int64) * DEG, M).astype(np.int32)
    w = np.random.default_rng(31).integers(1, 256, size=M, dtype=np.uint32)
    log("  max size: oracle ALIAS tables")
    thr, alias = oracle.alias_build(row_ptr, w)
    log("  max size: device graph, validation and ALIAS table")
    G = trw.Graph(row_ptr, col, w)
    assert G.validate() == 0
    table = G.table("alias")
    torch.cuda.synchronize()
    yield trw, G, table, row_ptr, col, w, thr, alias
    G.close()
    torch.cuda.empty_cache()


def _sources(k, seed):
    rng = np.random.default_rng(seed)
    tail = np.arange(N - 64, N, dtype=np.int32)                  # rows whose slots end at 2^31 - 1
    return np.concatenate([tail, rng.integers(0, N, k).astype(np.int32), np.array([0, N, -1], np.int32)])


def test_alias_entries_at_both_ends(big):
    trw, G, table, row_ptr, col, w, thr, alias = big
    raw = table.buf.view(torch.int32)
    for v in (0, 1, N // 2, N - 2, N - 1):
        a, b = int(row_ptr[v]), int(row_ptr[v + 1])
        ent = raw[8 * a:8 * b].cpu().numpy().view(np.uint32).reshape(-1, 8)
        first, second = col[a:b], col[a + alias[a:b]]
        assert np.array_equal(ent[:, 0], thr[a:b]), v
        assert np.array_equal(ent[:, 1].view(np.int32), first), v
        assert np.array_equal(ent[:, 2].view(np.int32), second), v
        for k, x in ((4, first), (6, second)):     # the candidates' row ranges, up to 2^31 - 1
            assert np.array_equal(ent[:, k].view(np.int32), row_ptr[x]), v
            assert np.array_equal(ent[:, k + 1].view(np.int32), row_ptr[x + 1] - row_ptr[x]), v


def test_ppr_alias_at_max_size(big):
    trw, G, table, row_ptr, col, w, thr, alias = big
    src = _sources(3000, 32)
    stop = oracle.stop_q32(0.2)
    log(f"  max size: PPR ALIAS, {len(src)} queries")
    p = trw.make_params("ppr", "alias", 256, 33, stop_q32=stop)
    P, L, S = trw.walk(G, table, p, torch.from_numpy(src).cuda())
    torch.cuda.synchronize()
    ref = oracle.walk(row_ptr, col, oracle.WalkParams(oracle.PPR, oracle.ALIAS, 256, 33, stop_q32=stop), src,
                      thr=thr, alias=alias)
    _check(P, L, S, ref, 256)


def test_deepwalk_naive_at_max_size(big):
    trw, G, table, row_ptr, col, w, thr, alias = big
    src = _sources(2000, 34)
    log(f"  max size: DeepWalk NAIVE, {len(src)} queries")
    p = trw.make_params("deepwalk", "naive", 40, 35)
    P, L, S = trw.walk(G, None, p, torch.from_numpy(src).cuda())
    torch.cuda.synchronize()
    ref = oracle.walk(row_ptr, col, oracle.WalkParams(oracle.DEEPWALK, oracle.NAIVE, 40, 35), src)
    _check(P, L, S, ref, 40)


def _check(P, L, S, ref, max_len):
    gp, gl, gs = P.cpu().numpy(), L.cpu().numpy().view(np.uint32), S.cpu().numpy()
    assert np.array_equal(gs, ref.status)
    assert np.array_equal(gl, ref.lengths)
    ok = ref.status != oracle.ST_BAD_SOURCE
    mask = (np.arange(max_len + 1)[None, :] <= ref.lengths[:, None]) & ok[:, None]
    assert not ((gp[:, :max_len + 1] != ref.paths) & mask).any()
    assert (ref.status == oracle.ST_BAD_SOURCE).sum() == 2


def test_counting_walk_at_max_queries():
    """nq = 2^32 - 1, the most one call takes: query indices reach one below the value that marks an
    idle lane.  The counting walk stores no per-query outputs, so the batch is the sources (17 GB) and
    the counts.  The counts sum to nq, and the last group's counts equal the oracle's."""
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.empty_cache()                        # what earlier tests left in torch's cache
    free, _ = torch.cuda.mem_get_info()
    if free < 40 * (1 << 30):
        pytest.skip(f"needs ~40 GB of free device memory, {free >> 30} GB free")
    import paper_2107_11983_amd as trw
    import synth
    g = synth.attach_attrs(synth.rmat(16, 16, False, 0x3A7), 0x3A8, weights=True)
    G = trw.Graph(g.row_ptr, g.col, g.weight)
    table = G.table("alias")
    nq, group = (1 << 32) - 1, 1 << 20
    log(f"  max queries: {nq} sources on the device")
    src = torch.empty(nq, dtype=torch.int32, device="cuda")
    step = 1 << 27
    for c in range(0, nq, step):
        idx = torch.arange(c, min(nq, c + step), dtype=torch.int64, device="cuda")
        src[c:c + idx.numel()] = ((idx * 40503 + 17) % g.n).to(torch.int32)
    del idx
    stop = oracle.stop_q32(0.2)
    p = trw.make_params("ppr", "alias", 256, 36, stop_q32=stop)
    log("  max queries: counting walk")
    counts, L, S = trw.ppr_walk_counts(G, table, p, src, group=group, outputs=False)
    torch.cuda.synchronize()
    assert L is None and counts.shape == (-(-nq // group), g.n)
    assert int(counts.to(torch.int64).sum().item()) == nq
    first = (nq // group) * group
    last_src = ((np.arange(first, nq, dtype=np.int64) * 40503 + 17) % g.n).astype(np.int32)
    log(f"  max queries: oracle on the last {nq - first} queries")
    thr, alias = oracle.alias_build(g.row_ptr, g.weight)
    ref = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.PPR, oracle.ALIAS, 256, 36, stop_q32=stop),
                      last_src, qid_base=first, thr=thr, alias=alias)
    exp, skipped = oracle.end_counts(g.n, ref.paths, ref.lengths, ref.status)
    assert skipped == 0
    assert np.array_equal(counts[-1].cpu().numpy().view(np.uint32), exp[0])
    del src, counts
    G.close()
    torch.cuda.empty_cache()
