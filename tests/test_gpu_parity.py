"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Tables: ALIAS entries and ITS prefixes equal the oracle's, slot by slot.
Walks: lengths, status and every path entry equal the oracle's for every
(algorithm, sampler) pair, both schedules and every walkers-per-lane setting,
on inputs that span many waves and end in a ragged tail, plus edge cases.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import star, undirected, zoo

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
    sys.stdout.flush()


ORC_ALGO = {"deepwalk": oracle.DEEPWALK, "ppr": oracle.PPR, "node2vec": oracle.NODE2VEC, "metapath": oracle.METAPATH}
ORC_SMP = {"naive": oracle.NAIVE, "alias": oracle.ALIAS, "its": oracle.ITS, "orej": oracle.OREJ, "rej": oracle.REJ}


class Case:
    """A host graph, its device twin and the oracle's tables."""

    def __init__(self, g, symmetric=False):
        self.g = g
        self.G = trw.Graph(g.row_ptr, g.col, g.weight, g.label, symmetric=symmetric)
        assert self.G.validate() == 0
        self._dev_tables = {}
        self._orc_tables = {}

    def dev_table(self, sampler):
        if sampler not in ("alias", "its", "rej"):
            return None
        if sampler not in self._dev_tables:
            self._dev_tables[sampler] = self.G.table(sampler)
        return self._dev_tables[sampler]

    def adjacency_index(self):
        if "adj" not in self._dev_tables:
            self._dev_tables["adj"] = self.G.adjacency_index()
        return self._dev_tables["adj"]

    def edge_index(self):
        if "eidx" not in self._dev_tables:
            self._dev_tables["eidx"] = self.G.edge_index()
        return self._dev_tables["eidx"]

    def label_index(self, n_labels):
        key = ("label_index", n_labels)
        if key not in self._dev_tables:
            self._dev_tables[key] = self.G.label_index(n_labels)
        return self._dev_tables[key]

    def orc_tables(self, sampler):
        if sampler not in self._orc_tables:
            if sampler == "alias":
                t, a = oracle.alias_build(self.g.row_ptr, self.g.weight)
                self._orc_tables[sampler] = dict(thr=t, alias=a)
            elif sampler == "its":
                self._orc_tables[sampler] = dict(prefix=oracle.its_build(self.g.row_ptr, self.g.weight))
            elif sampler == "rej":
                self._orc_tables[sampler] = dict(weight=self.g.weight,
                                                 pmax=oracle.rej_build(self.g.row_ptr, self.g.weight))
            else:
                self._orc_tables[sampler] = {}
        return self._orc_tables[sampler]


def run_both(case, algo, sampler, max_len, seed, src, mode, tuning=None, qid_base=0, stop=0,
             thr=(65536, 65536, 65536), schema=(), stride=0, label_index=0, adjacency=False, edge_index=False):
    g = case.g
    src = np.ascontiguousarray(src, dtype=np.int32)
    nq = len(src)
    log(f"  walk {algo}/{sampler} mode={mode} nq={nq} max_len={max_len} tuning={tuning and tuning.as_dict()}")
    p = trw.make_params(algo, sampler, max_len, seed, stop_q32=stop, n2v_thr_q16=thr, schema=schema)
    bufs = trw.WalkBuffers(case.G, p, nq, mode, stride)
    bufs.paths.fill_(-7)
    d_src = torch.from_numpy(src).cuda()
    table = case.dev_table(sampler) if algo in ("deepwalk", "ppr") else None
    if algo == "metapath" and label_index:
        table = case.label_index(label_index)
    if edge_index:
        assert sampler in ("naive", "orej")
        table = case.edge_index()
    if adjacency:
        assert sampler in ("naive", "orej")
        table = case.adjacency_index()
    trw.walk(case.G, table, p, d_src, qid_base=qid_base, mode=mode, tuning=tuning, bufs=bufs)
    torch.cuda.synchronize()
    gp = bufs.paths.cpu().numpy()
    gl = bufs.lengths.cpu().numpy().view(np.uint32)
    gs = bufs.status.cpu().numpy()
    kw = dict(case.orc_tables(sampler)) if algo in ("deepwalk", "ppr") else {}
    if algo == "metapath":
        kw["label"] = g.label
    op = oracle.WalkParams(ORC_ALGO[algo], ORC_SMP[sampler], max_len, seed, stop_q32=stop,
                           n2v_thr_q16=tuple(thr), schema=tuple(schema))
    ref = oracle.walk(g.row_ptr, g.col, op, src, qid_base=qid_base, **kw)
    return (gp, gl, gs), ref


def assert_same(gpu, ref, max_len):
    gp, gl, gs = gpu
    assert np.array_equal(gs, ref.status), f"status differs at {np.nonzero(gs != ref.status)[0][:10]}"
    assert np.array_equal(gl, ref.lengths), f"lengths differ at {np.nonzero(gl != ref.lengths)[0][:10]}"
    ok = ref.status != oracle.ST_BAD_SOURCE
    mask = (np.arange(max_len + 1)[None, :] <= ref.lengths[:, None]) & ok[:, None]
    bad = np.nonzero((gp[:, :max_len + 1] != ref.paths) & mask)
    assert bad[0].size == 0, f"paths differ at queries {np.unique(bad[0])[:10]}"
    # rows of bad sources are left untouched
    if (~ok).any():
        assert (gp[~ok] == -7).all()


# --------------------------------------------------------------------------- fixtures
@pytest.fixture(scope="module")
def rmat_sym():
    g = synth.rmat(11, 12, True, 0xC0FFEE)
    synth.attach_attrs(g, 0xC0FFEE ^ 3, weights=True, labels=5)
    return Case(g, symmetric=True)


@pytest.fixture(scope="module")
def rmat_dir():
    g = synth.rmat(11, 16, False, 0xD1CE)
    synth.attach_attrs(g, 0xD1CE ^ 3, weights=True)
    return Case(g)


# --------------------------------------------------------------------------- tables
def _alias_expected(g, thr, alias):
    """The documented 32-byte ALIAS entry for every edge slot, from the oracle's (thr, alias)."""
    rp, col = g.row_ptr.astype(np.int64), g.col.astype(np.int64)
    m = g.m
    exp = np.zeros((m, 8), dtype=np.int64)
    src_row = np.repeat(np.arange(g.n), np.diff(rp))
    dead = alias < 0
    second = np.where(dead, -1, col[np.clip(rp[src_row] + alias, 0, max(m - 1, 0))])
    first = np.where(dead, -1, col)
    deg = np.diff(rp)
    exp[:, 0] = thr
    exp[:, 1] = first
    exp[:, 2] = second
    exp[:, 4] = np.where(dead, 0, rp[np.clip(first, 0, None)])
    exp[:, 5] = np.where(dead, 0, deg[np.clip(first, 0, None)])
    exp[:, 6] = np.where(dead, 0, rp[np.clip(second, 0, None)])
    exp[:, 7] = np.where(dead, 0, deg[np.clip(second, 0, None)])
    return (exp & 0xFFFFFFFF).astype(np.uint32)


def _alias_got(t, m):
    return t.buf[:32 * m].view(torch.int32).cpu().numpy().view(np.uint32).reshape(-1, 8)


def _weighted_rows_graph(seed, wmax, zero_rows=True):
    rng = np.random.default_rng(seed)
    edges, ws = [], []
    n = 300
    for v in range(n):
        d = int(rng.integers(0, 120)) if v % 7 else int(rng.integers(300, 2000))
        d = min(d, n - 1)
        nb = np.sort(rng.choice(np.setdiff1d(np.arange(n), [v]), size=d, replace=False))
        w = rng.integers(1, wmax + 1, size=d, dtype=np.uint64).astype(np.uint32)
        if zero_rows and v % 11 == 0:
            w[:] = 0
        elif zero_rows and v % 5 == 0 and d > 2:
            w[::2] = 0
        edges += [(v, int(x)) for x in nb]
        ws += w.tolist()
    return synth.from_edges(n, edges, ws)


@pytest.mark.parametrize("wmax", [255, 2**32 - 1])
def test_alias_table_matches_oracle(wmax):
    g = _weighted_rows_graph(wmax % 1000, wmax)
    case = Case(g)
    log(f"  alias table m={g.m}")
    t = case.dev_table("alias")
    torch.cuda.synchronize()
    got = _alias_got(t, g.m)
    thr, alias = oracle.alias_build(g.row_ptr, g.weight)
    exp = _alias_expected(g, thr, alias)
    bad = np.nonzero((got != exp).any(axis=1))[0]
    assert bad.size == 0, f"alias entries differ at edge slots {bad[:10]}"


def test_alias_table_rmat(rmat_dir):
    g = rmat_dir.g
    t = rmat_dir.dev_table("alias")
    torch.cuda.synchronize()
    got = _alias_got(t, g.m)
    thr, alias = oracle.alias_build(g.row_ptr, g.weight)
    assert np.array_equal(got, _alias_expected(g, thr, alias))


def _its_check(case):
    """The documented ITS table: the oracle's prefix, then per slot {dst, row(dst), W(dst)}, then W[n]."""
    g = case.g
    t = case.dev_table("its")
    torch.cuda.synchronize()
    raw = t.buf.cpu().numpy()
    prefix = oracle.its_build(g.row_ptr, g.weight)
    assert np.array_equal(raw[:8 * g.m].view(np.uint64), prefix)
    rp = g.row_ptr.astype(np.int64)
    deg = np.diff(rp)
    W = np.where(deg > 0, prefix[np.clip(rp[1:] - 1, 0, None)] if g.m else 0, 0).astype(np.uint64)
    pb = (8 * g.m + 255) // 256 * 256
    nb = (32 * g.m + 255) // 256 * 256
    assert np.array_equal(raw[pb + nb:pb + nb + 8 * g.n].view(np.uint64), W), "W[n] differs"
    rec = raw[pb:pb + 32 * g.m].view(np.uint32).reshape(-1, 8)
    col = g.col.astype(np.int64)
    exp = np.zeros((g.m, 8), np.uint64)
    exp[:, 0] = col
    exp[:, 1] = rp[col]
    exp[:, 2] = deg[col]
    exp[:, 4] = W[col] & np.uint64(0xFFFFFFFF)
    exp[:, 5] = W[col] >> np.uint64(32)
    bad = np.nonzero((rec != exp.astype(np.uint32)).any(axis=1))[0]
    assert bad.size == 0, f"ITS records differ at edge slots {bad[:10]}"


def test_its_table_matches_oracle(rmat_dir):
    for case in (rmat_dir, Case(_weighted_rows_graph(5, 2**32 - 1))):
        _its_check(case)


def _rej_expected(g, pmax):
    """The documented REJ table: 32-byte slot records, then p*[n] at 32*m rounded to 256."""
    rp, col = g.row_ptr.astype(np.int64), g.col.astype(np.int64)
    deg = np.diff(rp)
    exp = np.zeros((g.m, 8), dtype=np.int64)
    exp[:, 0] = g.weight
    exp[:, 1] = col
    exp[:, 2] = rp[col]
    exp[:, 3] = deg[col]
    exp[:, 4] = pmax[col]
    return exp.astype(np.uint32)


def _rej_check(case):
    g = case.g
    t = case.dev_table("rej")
    torch.cuda.synchronize()
    raw = t.buf.view(torch.int32).cpu().numpy().view(np.uint32)
    pmax = oracle.rej_build(g.row_ptr, g.weight)
    rec_words = ((32 * g.m + 255) // 256 * 256) // 4
    assert np.array_equal(raw[rec_words:rec_words + g.n], pmax), "p* differs"
    got = raw[:8 * g.m].reshape(-1, 8)
    bad = np.nonzero((got != _rej_expected(g, pmax)).any(axis=1))[0]
    assert bad.size == 0, f"REJ records differ at edge slots {bad[:10]}"


def test_rej_table_matches_oracle(rmat_dir):
    _rej_check(rmat_dir)
    _rej_check(Case(_weighted_rows_graph(9, 2**32 - 1)))


def _long_rows_graph(wmax, seed):
    """Rows of 1025..5000 slots (one workgroup each) in every weight regime, a
    70000-slot star whose d*W passes 2^64 at wmax = 2^32-1, and short rows."""
    rng = np.random.default_rng(seed)
    n = 70001
    edges, ws = [], []
    for v in range(24):
        d = int(rng.integers(1025, 5000)) if v % 4 else int(rng.integers(1, 1025))
        nb = np.sort(rng.choice(np.arange(24, n), size=d, replace=False))
        kind = v % 6
        if kind == 0:
            w = rng.integers(1, wmax + 1, size=d, dtype=np.uint64)
        elif kind == 1:
            w = np.full(d, min(wmax, 77), np.uint64)                 # every bucket full
        elif kind == 2:
            w = (rng.random(d) < 0.02) * rng.integers(1, wmax + 1, size=d, dtype=np.uint64)
        elif kind == 3:
            w = np.ones(d, np.uint64); w[int(rng.integers(0, d))] = wmax   # one dominant column
        elif kind == 4:
            w = np.zeros(d, np.uint64)                               # no transition
        else:
            w = rng.integers(0, 3, size=d).astype(np.uint64)
        if not w.any() and kind != 4:
            w[0] = 1
        edges += [(v, int(x)) for x in nb]
        ws += w.astype(np.uint32).tolist()
    star = n - 1
    for x in range(n - 1):
        edges.append((star, x))
        ws.append(int(rng.integers(wmax - wmax // 16, wmax + 1)))
    for x in range(24, 3000):
        edges.append((x, int(rng.integers(0, 24))))
        ws.append(int(rng.integers(1, wmax + 1)))
    return synth.from_edges(n, edges, ws)


@pytest.mark.parametrize("wmax", [255, 2**32 - 1])
def test_tables_long_rows(wmax):
    g = _long_rows_graph(wmax, 41 + (wmax & 7))
    case = Case(g)
    log(f"  long-row tables m={g.m} max_deg={int(np.diff(g.row_ptr).max())}")
    t = case.dev_table("alias")
    torch.cuda.synchronize()
    thr, alias = oracle.alias_build(g.row_ptr, g.weight)
    bad = np.nonzero((_alias_got(t, g.m) != _alias_expected(g, thr, alias)).any(axis=1))[0]
    assert bad.size == 0, f"alias entries differ at edge slots {bad[:10]}"
    _its_check(case)
    _rej_check(case)


def test_label_index_records_long_rows():
    """Label index of rows up to 6000 slots: per-label offsets and a stable sort by label."""
    rng = np.random.default_rng(12)
    n, L = 8000, 5
    edges, labs = [], []
    for v in range(n):
        d = int(rng.integers(1025, 6000)) if v < 12 else int(rng.integers(0, 6))
        nb = np.sort(rng.choice(n, size=d, replace=False))
        edges += [(v, int(x)) for x in nb if x != v]
    labs = rng.integers(0, L + 2, size=len(edges)).tolist()   # some labels >= L stay out
    g = synth.from_edges(n, edges, labels=labs)
    case = Case(g)
    t = case.label_index(L)
    torch.cuda.synchronize()
    raw = t.buf.view(torch.int32).cpu().numpy()
    head = n * (L + 1)
    pad = ((head * 4 + 255) // 256) * 256 // 4
    loff = raw[:head].reshape(n, L + 1)
    lcol = raw[pad:pad + g.m]
    rp = g.row_ptr.astype(np.int64)
    lab = g.label.astype(np.int64)
    for v in range(n):
        a, b = rp[v], rp[v + 1]
        pos = a
        for x in range(L):
            assert loff[v, x] == pos, (v, x)
            sel = g.col[a:b][lab[a:b] == x]
            assert np.array_equal(lcol[pos:pos + sel.size], sel), (v, x)
            pos += sel.size
        assert loff[v, L] == pos
        assert (lcol[pos:b] == -1).all()
    # L <= 6: fused entries {lcol[e], loff[lcol[e]][0..L], 0...} after lcol, 256-byte aligned
    fpad = pad + ((g.m * 4 + 255) // 256) * 256 // 4
    fused = raw[fpad:fpad + 8 * g.m].reshape(g.m, 8)
    assert np.array_equal(fused[:, 0], lcol)
    ok = lcol >= 0
    assert np.array_equal(fused[ok, 1:L + 2], loff[lcol[ok]])
    assert (fused[ok, L + 2:] == 0).all() and (fused[~ok, 1:] == 0).all()


def test_validate_rejects_bad_graphs():
    g = synth.from_edges(4, [(0, 1), (0, 2), (1, 0), (2, 3)])
    G = trw.Graph(g.row_ptr, g.col)
    assert G.validate() == 0
    bad_col = g.col.copy()
    bad_col[0], bad_col[1] = bad_col[1], bad_col[0]          # unsorted row
    assert trw.Graph(g.row_ptr, bad_col).validate() == 1
    bad_col2 = g.col.copy()
    bad_col2[3] = 9                                          # out of range
    assert trw.Graph(g.row_ptr, bad_col2).validate() >= 1
    dup = synth.from_edges(3, [(0, 1), (0, 1), (1, 2)])      # duplicate edge
    assert trw.Graph(dup.row_ptr, dup.col).validate() == 1


# --------------------------------------------------------------------------- walks
PAIRS = [("deepwalk", "naive"), ("deepwalk", "alias"), ("deepwalk", "its"), ("deepwalk", "rej"),
         ("ppr", "naive"), ("ppr", "alias"), ("ppr", "its"), ("ppr", "rej"),
         ("node2vec", "orej"), ("metapath", "its")]


def _args(algo):
    kw = {}
    if algo == "ppr":
        kw["stop"] = oracle.stop_q32(0.2)
    if algo == "node2vec":
        kw["thr"] = oracle.n2v_thresholds(2.0, 0.5)
    if algo == "metapath":
        kw["schema"] = (3, 1, 4, 1, 0)
    return kw


@pytest.mark.parametrize("algo,sampler", PAIRS)
@pytest.mark.parametrize("mode", [1, 0])
def test_walk_parity(rmat_sym, rmat_dir, algo, sampler, mode):
    case = rmat_dir if algo == "ppr" else rmat_sym
    n = case.g.n
    src = np.concatenate([np.arange(n), synth.sources(37 + 64 * 3, n, 4)]).astype(np.int32)  # ragged tail
    max_len = 256 if algo == "ppr" else (100 if algo == "metapath" else 40)
    gpu, ref = run_both(case, algo, sampler, max_len, 0x5EED + mode, src, mode, **_args(algo))
    assert_same(gpu, ref, max_len)
    assert ref.counters["moves"] > 0


@pytest.mark.parametrize("algo,sampler", [("ppr", "alias"), ("node2vec", "orej"), ("metapath", "its"),
                                          ("deepwalk", "its"), ("ppr", "rej")])
@pytest.mark.parametrize("wpl,bpc,chunk,threads", [(2, 8, 256, 256), (4, 4, 64, 256), (1, 1, 1, 64),
                                                   (2, 3, 1000, 128)])
def test_tuning_does_not_change_results(rmat_sym, rmat_dir, algo, sampler, wpl, bpc, chunk, threads):
    case = rmat_dir if algo == "ppr" else rmat_sym
    src = synth.sources(3 * 1024 + 5, case.g.n, 99)
    max_len = 64
    tu = trw.make_tuning(walkers_per_lane=wpl, blocks_per_cu=bpc, queue_chunk=chunk, block_threads=threads)
    gpu, ref = run_both(case, algo, sampler, max_len, 77, src, 1, tuning=tu, **_args(algo))
    assert_same(gpu, ref, max_len)



@pytest.mark.parametrize("algo,sampler,index", [("ppr", "alias", None), ("metapath", "its", None),
                                                ("node2vec", "orej", "adj"), ("node2vec", "orej", "eidx"),
                                                ("ppr", "its", None)])
def test_autotune_picks_a_candidate_and_results_do_not_change(rmat_sym, rmat_dir, algo, sampler, index):
    case = rmat_dir if algo == "ppr" else rmat_sym
    src = synth.sources(20000, case.g.n, 31)
    kw = _args(algo)
    p = trw.make_params(algo, sampler, 40, 9, stop_q32=kw.get("stop", 0), n2v_thr_q16=kw.get("thr", (65536,) * 3),
                        schema=kw.get("schema", ()))
    table = case.dev_table(sampler) if algo == "ppr" else (
        case.adjacency_index() if index == "adj" else case.edge_index() if index == "eidx" else None)
    d_src = torch.from_numpy(src).cuda()
    best, ms = trw.autotune(case.G, table, p, d_src, mode=trw.TRW_M_PERSISTENT)
    assert ms > 0 and best.walkers_per_lane in (1, 2, 4) and best.blocks_per_cu >= 1
    ref = [x.cpu().numpy() for x in trw.walk(case.G, table, p, d_src)]
    got = [x.cpu().numpy() for x in trw.walk(case.G, table, p, d_src, tuning=best)]
    L = ref[1].view(np.uint32)
    assert np.array_equal(ref[1], got[1]) and np.array_equal(ref[2], got[2])
    mask = np.arange(41)[None, :] <= L[:, None]
    assert np.array_equal(ref[0][:, :41][mask], got[0][:, :41][mask])

@pytest.mark.parametrize("mode", [1, 0])
@pytest.mark.parametrize("algo", ["deepwalk", "ppr"])
@pytest.mark.parametrize("sampler", ["rej", "its", "alias"])
def test_weighted_walk_zero_weights_and_long_rows(sampler, algo, mode):
    """Weighted samplers where rows have zero weights (dead ends), skewed
    weights (many REJ misses, deep ITS searches) and thousands of slots."""
    for case in (Case(_weighted_rows_graph(17, 255)), Case(_long_rows_graph(2**32 - 1, 5))):
        n = case.g.n
        src = np.concatenate([np.arange(min(n, 3000)), synth.sources(1000 + 29, n, 8)]).astype(np.int32)
        max_len = 30
        gpu, ref = run_both(case, algo, sampler, max_len, 21 + mode, src, mode, **_args(algo))
        assert_same(gpu, ref, max_len)
        if sampler == "rej":
            assert ref.counters["rej_trials"] > ref.counters["moves"]   # darts did miss


def test_edge_cases(rmat_sym, rmat_dir):
    n = rmat_dir.g.n
    deg = rmat_dir.g.degrees()
    dangling = np.nonzero(deg == 0)[0][:5]
    assert len(dangling) > 0
    # bad sources, dangling sources, one query, qid offset, wide stride
    src = np.array([0, -1, n, int(dangling[0]), 5, 2**31 - 1, int(dangling[-1]), 7], np.int32)
    for mode in (1, 0):
        for algo, sampler in PAIRS:
            case = rmat_dir if algo == "ppr" else rmat_sym
            gpu, ref = run_both(case, algo, sampler, 9, 3, src, mode, qid_base=(1 << 40) + 5, stride=13,
                                **_args(algo))
            assert_same(gpu, ref, 9)
        gpu, ref = run_both(rmat_dir, "ppr", "alias", 1, 3, src[4:5], mode)
        assert_same(gpu, ref, 1)
        gpu, ref = run_both(rmat_sym, "deepwalk", "naive", 1, 3, np.arange(n, dtype=np.int32), mode)
        assert_same(gpu, ref, 1)



def test_validate_sources(rmat_dir):
    """trw_validate_sources counts the sources outside [0, n) exactly (TRW_E_INVALID when any)."""
    import ctypes
    from paper_2107_11983_amd import _abi
    G = rmat_dir.G
    n = rmat_dir.g.n
    ws = torch.empty(8, dtype=torch.int64, device="cuda")
    rng = np.random.default_rng(11)
    edge = np.array([0, n - 1, n, -1, -2**31, 2**31 - 1, n + 1, 1], np.int32)
    big = rng.integers(0, n, size=5_000_017, dtype=np.int64).astype(np.int32)
    where = rng.choice(big.size, size=1234, replace=False)
    big[where] = rng.choice([-1, n, 2**31 - 1, -2**31], size=where.size)
    cases = [np.zeros(0, np.int32), np.arange(n, dtype=np.int32), edge, big, np.full(1000, -7, np.int32)]
    for src in cases:
        expect = int(((src < 0) | (src >= n)).sum())
        d = torch.from_numpy(src).cuda() if src.size else torch.zeros(1, dtype=torch.int32, device="cuda")
        bad = ctypes.c_uint64(12345)
        st = _abi.trw_validate_sources(G.handle, ctypes.c_void_p(d.data_ptr()), int(src.size),
                                       ctypes.c_void_p(ws.data_ptr()), 8, None, ctypes.byref(bad))
        assert int(bad.value) == expect, (src.size, int(bad.value), expect)
        assert st == (_abi.TRW_E_INVALID if expect else _abi.TRW_OK)
        assert G.validate_sources(d[:src.size]) == expect
    log(f"  validate_sources: {len(cases)} arrays counted exactly")


@pytest.mark.parametrize("stride", [13, 16, 20, 81])
def test_path_padding_stays_in_row(rmat_dir, stride):
    """A walk may fill the rest of its last 64-byte block with -1, but only
    inside its own row: other rows and the memory after the last row keep
    their contents, and the paths still equal the oracle's."""
    case = rmat_dir
    g = case.g
    src = synth.sources(5000, g.n, 12)
    p = trw.make_params("ppr", "alias", 12, 5, stop_q32=trw.stop_threshold(0.2))
    ref = oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.PPR, oracle.ALIAS, 12, 5, stop_q32=p.stop_q32),
                      src, **case.orc_tables("alias"))
    sentinel = 0x7EEEEEEE
    for mode in (1, 0):
        bufs = trw.WalkBuffers(case.G, p, len(src), mode, stride)
        big = torch.full((len(src) + 3, stride), sentinel, dtype=torch.int32, device="cuda")
        bufs.paths = big[:len(src)]
        _, L, S = trw.walk(case.G, case.dev_table("alias"), p, torch.from_numpy(src).cuda(), mode=mode, bufs=bufs)
        torch.cuda.synchronize()
        B = big.cpu().numpy()
        L = L.cpu().numpy().view(np.uint32)
        assert (B[len(src):] == sentinel).all(), "writes past the last row"
        assert np.array_equal(L, ref.lengths) and np.array_equal(S.cpu().numpy(), ref.status)
        inside = np.arange(stride)[None, :] <= L[:, None]
        assert np.array_equal(B[:len(src), :13][inside[:, :13]], ref.paths[inside[:, :13]])
        past = B[:len(src)][~inside]
        assert np.isin(past, [sentinel, -1]).all(), "a row's entries past its end hold another row's data"

def test_zero_weight_rows_are_dead_ends():
    g = _weighted_rows_graph(9, 255)
    case = Case(g)
    src = np.arange(g.n, dtype=np.int32)
    for sampler in ("alias", "its"):
        for mode in (1, 0):
            gpu, ref = run_both(case, "deepwalk", sampler, 30, 11, src, mode)
            assert_same(gpu, ref, 30)
            assert (ref.status == oracle.ST_DEAD_END).any()


def test_zoo_graphs():
    for name, g in zoo().items():
        case = Case(g, symmetric=True)
        src = np.tile(np.arange(g.n, dtype=np.int32), 50)
        for algo, sampler in PAIRS:
            gpu, ref = run_both(case, algo, sampler, 12, 5, src, 1, **_args(algo))
            assert_same(gpu, ref, 12)


def test_longest_walk():
    n = 5
    g = synth.from_edges(n, [(i, (i + 1) % n) for i in range(n)], weights=[2] * n)
    case = Case(g)
    src = np.array([0, 3], np.int32)
    for mode in (1, 0):
        gpu, ref = run_both(case, "deepwalk", "alias", 65535, 1, src, mode)
        assert_same(gpu, ref, 65535)
        assert (ref.lengths == 65535).all()


def test_empty_batch(rmat_sym):
    p = trw.make_params("deepwalk", "naive", 5, 1)
    bufs = trw.WalkBuffers(rmat_sym.G, p, 0, 1)
    trw.walk(rmat_sym.G, None, p, torch.empty(0, dtype=torch.int32, device="cuda"), bufs=bufs)
    torch.cuda.synchronize()


# --------------------------------------------------------------------------- workloads
def test_deepwalk_rmat12_full():
    """DeepWalk on the 2^12-vertex symmetric R-MAT graph, one walk of 80 per vertex."""
    wl = synth.WORKLOADS["deepwalk-rmat12"]
    g = synth.make_graph(wl)
    case = Case(g, symmetric=True)
    src = synth.make_sources(wl, g)
    for mode in (1, 0):
        for adjacency in (False, True):          # bench.py times the adjacency index
            gpu, ref = run_both(case, "deepwalk", "naive", 80, wl.walk_seed, src, mode, adjacency=adjacency)
            assert_same(gpu, ref, 80)


@pytest.mark.parametrize("name", ["ppr-rmat22", "node2vec-rmat24", "metapath-rmat24"])
def test_workloads_reduced_scale(name):
    """The larger workloads' recipes at 2^16 vertices, compared in full."""
    wl = synth.WORKLOADS[name]
    g = synth.make_graph(wl, scale=16)
    case = Case(g, symmetric=wl.symmetric)
    src = synth.make_sources(wl, g, nq=200_000 if wl.nq else None)
    kw = _args(wl.algo)
    if wl.algo == "metapath":
        kw["schema"] = tuple(int(x) for x in synth.make_schema(wl))
    for sampler in wl.samplers:
        for mode in (1, 0):
            gpu, ref = run_both(case, wl.algo, sampler, wl.max_len, wl.walk_seed, src, mode, **kw)
            assert_same(gpu, ref, wl.max_len)
            if wl.algo == "metapath":
                gpu, ref = run_both(case, wl.algo, sampler, wl.max_len, wl.walk_seed, src, mode,
                                    label_index=wl.labels, **kw)
                assert_same(gpu, ref, wl.max_len)
            if wl.algo == "node2vec":
                gpu, ref = run_both(case, wl.algo, sampler, wl.max_len, wl.walk_seed, src, mode,
                                    adjacency=True, **kw)
                assert_same(gpu, ref, wl.max_len)


# --------------------------------------------------------------------------- MetaPath gathers
@pytest.mark.parametrize("mode", [1, 0])
@pytest.mark.parametrize("n_labels", [5, 8])
def test_metapath_label_index(rmat_sym, mode, n_labels):
    n = rmat_sym.g.n
    src = np.concatenate([np.arange(n), synth.sources(301, n, 8)]).astype(np.int32)
    gpu, ref = run_both(rmat_sym, "metapath", "its", 100, 21, src, mode, schema=(3, 1, 4, 1, 0, 2, 2),
                        label_index=n_labels)
    assert_same(gpu, ref, 100)


@pytest.mark.parametrize("coop", [1, 3, 64, 1 << 30])
def test_metapath_cooperative_scan(rmat_sym, coop):
    n = rmat_sym.g.n
    src = np.arange(n, dtype=np.int32)
    for mode in (1, 0):
        tu = trw.make_tuning(coop_degree=coop)
        gpu, ref = run_both(rmat_sym, "metapath", "its", 60, 5, src, mode, tuning=tu, schema=(0, 4, 2))
        assert_same(gpu, ref, 60)


def test_metapath_hub_rows_unaligned():
    """Rows of 1..6000 labels at every byte alignment, labels to the end of the array."""
    rng = np.random.default_rng(3)
    edges, labs = [], []
    n = 6500
    for v in range(40):
        d = int(rng.integers(1, 6000)) if v % 3 else int(rng.integers(1, 9))
        nb = np.sort(rng.choice(np.arange(40, n), size=d, replace=False))
        edges += [(v, int(x)) for x in nb]
        labs += rng.integers(0, 4, size=d).tolist()
    for x in range(40, n):            # every leaf points back to a few hubs
        for h in (0, 1, 2):
            edges.append((x, h))
            labs.append(int(rng.integers(0, 4)))
    g = synth.from_edges(n, edges, labels=labs)
    case = Case(g)
    src = np.tile(np.arange(40, dtype=np.int32), 64)
    for coop in (1 << 30, 100, 1):
        for mode in (1, 0):
            tu = trw.make_tuning(coop_degree=coop)
            gpu, ref = run_both(case, "metapath", "its", 30, 17, src, mode, tuning=tu, schema=(1, 0, 3, 2))
            assert_same(gpu, ref, 30)
    gpu, ref = run_both(case, "metapath", "its", 30, 17, src, 1, schema=(1, 0, 3, 2), label_index=4)
    assert_same(gpu, ref, 30)


def test_metapath_label_index_rejects_large_schema_labels(rmat_sym):
    p = trw.make_params("metapath", "its", 10, 1, schema=(1, 6))
    src = torch.arange(10, dtype=torch.int32, device="cuda")
    with pytest.raises(trw.TrwError):
        trw.walk(rmat_sym.G, rmat_sym.label_index(5), p, src)


# --------------------------------------------------------------------------- adjacency index
def test_adjacency_index_records(rmat_dir):
    g = rmat_dir.g
    t = rmat_dir.adjacency_index()
    torch.cuda.synchronize()
    got = t.buf[:16 * g.m].view(torch.int32).cpu().numpy().view(np.uint32).reshape(-1, 4)
    rp = g.row_ptr.astype(np.int64)
    assert np.array_equal(got[:, 0], g.col.view(np.uint32))
    assert np.array_equal(got[:, 1], rp[g.col].astype(np.uint32))
    assert np.array_equal(got[:, 2], np.diff(rp)[g.col].astype(np.uint32))


@pytest.mark.parametrize("algo,sampler", [("deepwalk", "naive"), ("ppr", "naive"), ("node2vec", "orej")])
@pytest.mark.parametrize("mode", [1, 0])
def test_adjacency_index_parity(rmat_sym, rmat_dir, algo, sampler, mode):
    for case in (rmat_sym, rmat_dir):          # Node2Vec on the directed graph searches prev's row only
        n = case.g.n
        src = np.concatenate([np.arange(n), synth.sources(77, n, 2)]).astype(np.int32)
        for pq in ((2.0, 0.5), (0.25, 4.0)):
            kw = _args(algo)
            if algo == "node2vec":
                kw["thr"] = oracle.n2v_thresholds(*pq)
            gpu, ref = run_both(case, algo, sampler, 50, 1234, src, mode, adjacency=True, **kw)
            assert_same(gpu, ref, 50)
            if algo != "node2vec":
                break



@pytest.mark.parametrize("algo,sampler", [("deepwalk", "naive"), ("node2vec", "orej")])
@pytest.mark.parametrize("mode", [1, 0])
def test_edge_index_parity(rmat_sym, rmat_dir, algo, sampler, mode):
    """Node2Vec's adjacency test by the edge index's hash set: same paths as the
    oracle's binary search, on a symmetric and a directed graph (where the test
    must ask about prev -> x, not x -> prev)."""
    for case in (rmat_sym, rmat_dir):
        n = case.g.n
        src = np.concatenate([np.arange(n), synth.sources(77, n, 3)]).astype(np.int32)
        for pq in ((2.0, 0.5), (0.25, 4.0), (1.0, 1.0)):
            kw = _args(algo)
            if algo == "node2vec":
                kw["thr"] = oracle.n2v_thresholds(*pq)
            gpu, ref = run_both(case, algo, sampler, 50, 4321, src, mode, edge_index=True, **kw)
            assert_same(gpu, ref, 50)
            if algo != "node2vec":
                break


@pytest.mark.parametrize("mode", [1, 0])
@pytest.mark.parametrize("degree", [8, 64, 1 << 30])
def test_its_gallop_degree_does_not_change_results(rmat_sym, rmat_dir, degree, mode):
    """ITS rows below the tuned degree bisect the whole row instead of searching
    from the guessed slot (1 << 30: every row bisects); the slot is the same."""
    for algo, case in (("deepwalk", rmat_sym), ("ppr", rmat_dir)):
        n = case.g.n
        src = np.concatenate([np.arange(n), synth.sources(61, n, 8)]).astype(np.int32)
        tu = trw.make_tuning(its_gallop_degree=degree)
        gpu, ref = run_both(case, algo, "its", 48, 606, src, mode, tuning=tu, **_args(algo))
        assert_same(gpu, ref, 48)


@pytest.mark.parametrize("mode", [1, 0])
@pytest.mark.parametrize("degree", [4, 64, 1 << 30])
def test_n2v_search_degree_does_not_change_results(rmat_sym, rmat_dir, degree, mode):
    """Node2Vec with the edge index: rows of the previous vertex up to the tuned
    degree are searched instead of probing the hash set (1 << 30: every row);
    the same paths as the oracle, on a symmetric and a directed graph."""
    for case in (rmat_sym, rmat_dir):
        n = case.g.n
        src = np.concatenate([np.arange(n), synth.sources(53, n, 12)]).astype(np.int32)
        tu = trw.make_tuning(n2v_search_degree=degree)
        for pq in ((2.0, 0.5), (0.25, 4.0)):
            gpu, ref = run_both(case, "node2vec", "orej", 50, 808, src, mode, tuning=tu, edge_index=True,
                                thr=oracle.n2v_thresholds(*pq))
            assert_same(gpu, ref, 50)


def test_edge_index_layout(rmat_dir):
    """The documented layout: adjacency records, then a hash set holding exactly the edges."""
    g = rmat_dir.g
    t = rmat_dir.edge_index()
    torch.cuda.synchronize()
    raw = t.buf.cpu().numpy()
    rec_bytes = (16 * g.m + 255) // 256 * 256
    rec = raw[:16 * g.m].view(np.uint32).reshape(-1, 4)
    assert np.array_equal(rec[:, 0].view(np.int32), g.col)
    slots = 64
    while slots < 2 * g.m:
        slots *= 2
    keys = raw[rec_bytes:rec_bytes + 8 * slots].view(np.uint64)
    assert raw.size >= rec_bytes + 8 * slots
    full = keys[keys != np.uint64(0xFFFFFFFFFFFFFFFF)]
    src = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(g.row_ptr.astype(np.int64)))
    want = (src << np.uint64(32)) | g.col.astype(np.uint64)
    assert np.array_equal(np.sort(full), np.sort(want))


def test_validate_checks_symmetry():
    g = synth.from_edges(4, [(0, 1), (1, 0), (1, 2), (2, 1), (2, 3)])      # (2,3) has no reverse
    assert trw.Graph(g.row_ptr, g.col, symmetric=False).validate() == 0
    assert trw.Graph(g.row_ptr, g.col, symmetric=True).validate() == 1
