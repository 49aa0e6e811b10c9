"""Streamed output (trw_walk_stream) against the oracle: the chunks, put back
together, hold exactly the oracle's paths, lengths and status, whatever the
chunk size (one query, ragged, larger than the batch); a bad source has an
empty path; a chunk function that stops the stream ends it with
TRW_E_CANCELLED after that chunk."""
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
def graphs():
    gd = synth.rmat(12, 16, False, 0x57EA)
    synth.attach_attrs(gd, 0x57EA ^ 3, weights=True)
    gs = synth.rmat(11, 12, True, 0x57EB)
    return gd, gs


def _collect(G, table, p, src, chunk, qid_base=0):
    chunks = []
    n = trw.walk_stream(G, table, p, torch.from_numpy(src).cuda(), chunk, chunks.append, qid_base=qid_base)
    assert n == len(chunks)
    return chunks


def _check(chunks, ref, src, chunk, qid_base):
    nq = len(src)
    assert [c["nq"] for c in chunks] == [min(chunk, nq - i) for i in range(0, nq, chunk)]
    lo = 0
    for c in chunks:
        assert c["qid_base"] == qid_base + lo
        n = c["nq"]
        L, S, off, ent = c["lengths"], c["status"], c["offsets"], c["entries"]
        assert np.array_equal(L, ref.lengths[lo:lo + n]) and np.array_equal(S, ref.status[lo:lo + n])
        assert off[0] == 0 and len(ent) == off[n]
        for i in range(n):
            q = lo + i
            path = ent[off[i]:off[i + 1]]
            if ref.status[q] == oracle.ST_BAD_SOURCE:
                assert path.size == 0
            else:
                assert np.array_equal(path, ref.paths[q, :ref.lengths[q] + 1]), q
        lo += n
    assert lo == nq


@pytest.mark.parametrize("chunk", [1000, 4097, 1, 1 << 20])
def test_stream_ppr_alias(graphs, chunk):
    g, _ = graphs
    G = trw.Graph(g.row_ptr, g.col, g.weight)
    alias = G.table("alias")
    src = np.concatenate([synth.sources(10007 if chunk > 1 else 300, g.n, 5), np.array([-1, g.n], np.int32)])
    stop = oracle.stop_q32(0.2)
    p = trw.make_params("ppr", "alias", 256, 17, stop_q32=stop)
    log(f"  stream ppr/alias chunk={chunk} nq={len(src)}")
    chunks = _collect(G, alias, p, src, chunk, qid_base=77)
    thr, al = oracle.alias_build(g.row_ptr, g.weight)
    ref = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.PPR, oracle.ALIAS, 256, 17, stop_q32=stop), src,
                      qid_base=77, thr=thr, alias=al)
    _check(chunks, ref, src, chunk, 77)
    G.close()


@pytest.mark.parametrize("algo,sampler", [("deepwalk", "naive"), ("node2vec", "orej")])
def test_stream_long_walks(graphs, algo, sampler):
    _, g = graphs
    G = trw.Graph(g.row_ptr, g.col, symmetric=True)
    src = np.arange(g.n, dtype=np.int32)
    thr = oracle.n2v_thresholds(2.0, 0.5)
    p = trw.make_params(algo, sampler, 80, 23, n2v_thr_q16=thr)
    chunks = _collect(G, None, p, src, 333)
    ref = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.ALGOS[algo], oracle.SAMPLERS[sampler], 80, 23,
                                                          n2v_thr_q16=thr), src)
    _check(chunks, ref, src, 333, 0)
    G.close()


def test_stream_stop_and_empty(graphs):
    g, _ = graphs
    G = trw.Graph(g.row_ptr, g.col, g.weight)
    p = trw.make_params("ppr", "naive", 64, 3, stop_q32=oracle.stop_q32(0.2))
    src = torch.from_numpy(synth.sources(5000, g.n, 9)).cuda()
    seen = []

    def stop_after_two(c):
        seen.append(c["qid_base"])
        return len(seen) == 2

    with pytest.raises(trw.TrwError) as ei:
        trw.walk_stream(G, None, p, src, 1000, stop_after_two)
    assert ei.value.status == trw._abi.TRW_E_CANCELLED and seen == [0, 1000]
    assert trw.walk_stream(G, None, p, src[:0], 1000, seen.append) == 0
    G.close()


@pytest.mark.parametrize("chunk", [4097, 1 << 20])
def test_stream_to_disk(graphs, chunk, tmp_path):
    """The library's own file sink (trw_chunk_to_fd): the chunks written to disk
    while the next chunk walks, read back, hold exactly the oracle's walks."""
    g, _ = graphs
    G = trw.Graph(g.row_ptr, g.col, g.weight)
    alias = G.table("alias")
    src = np.concatenate([synth.sources(20011, g.n, 6), np.array([-3], np.int32)])
    stop = oracle.stop_q32(0.2)
    p = trw.make_params("ppr", "alias", 256, 19, stop_q32=stop)
    path = str(tmp_path / "walks.bin")
    log(f"  stream to disk chunk={chunk} nq={len(src)}")
    nbytes = trw.walk_stream_to_file(G, alias, p, torch.from_numpy(src).cuda(), chunk, path, qid_base=5)
    chunks = list(trw.read_stream_file(path))
    assert nbytes == sum(16 + 4 * c["nq"] + c["nq"] + (8 - c["nq"] % 8) % 8 + 8 * (c["nq"] + 1)
                         + 4 * len(c["entries"]) for c in chunks)
    thr, al = oracle.alias_build(g.row_ptr, g.weight)
    ref = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.PPR, oracle.ALIAS, 256, 19, stop_q32=stop), src,
                      qid_base=5, thr=thr, alias=al)
    _check(chunks, ref, src, chunk, 5)
    G.close()
