"""The C ABI library on a host without a GPU: it loads, exports every symbol
that include/trw.h declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trw.h")


def _declared_functions():
    import glob
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(trw_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def abi():
    from paper_2107_11983_amd import _abi
    return _abi


def test_exports_every_declared_symbol(abi):
    names = _declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(abi.lib, n), f"{n} declared in trw.h but not exported"
    assert set(names) <= set(abi._SIGS), "binding lacks a declared function"


def test_abi_version(abi):
    m = re.search(r"#define TRW_ABI_VERSION (\d+)u", open(HEADER).read())
    assert abi.trw_abi_version() == int(m.group(1))


def _fake_graph(abi, labels=False, weights=False):
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    st = abi.trw_graph_create(100, 1000, fake, fake, fake if weights else None, fake if labels else None,
                              0, ctypes.byref(h))
    assert st == abi.TRW_OK, abi.trw_last_error()
    return h


def test_graph_create_rejects_bad_sizes(abi):
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    assert abi.trw_graph_create(0, 10, fake, fake, None, None, 0, ctypes.byref(h)) == abi.TRW_E_INVALID
    assert b"n must be" in abi.trw_last_error()
    assert abi.trw_graph_create(10, -1, fake, fake, None, None, 0, ctypes.byref(h)) == abi.TRW_E_INVALID
    assert abi.trw_graph_create(10, 2**31, fake, fake, None, None, 0, ctypes.byref(h)) == abi.TRW_E_INVALID
    assert abi.trw_graph_create(10, 5, None, fake, None, None, 0, ctypes.byref(h)) == abi.TRW_E_INVALID
    assert abi.trw_graph_create(10, 5, fake, fake, None, None, 0, None) == abi.TRW_E_INVALID


def _params(abi, algo, sampler, max_len=10, thr=(65536, 65536, 65536), schema=()):
    from paper_2107_11983_amd import make_params
    return make_params(algo, sampler, max_len, 1, n2v_thr_q16=thr, schema=schema)


def test_param_validation(abi):
    g = _fake_graph(abi)
    sz = ctypes.c_size_t()
    def ws(p, nq=10, mode=1):
        return abi.trw_walk_workspace_bytes(g, ctypes.byref(p), nq, mode, ctypes.byref(sz))
    assert ws(_params(abi, "deepwalk", "naive")) == abi.TRW_OK
    assert ws(_params(abi, "deepwalk", "orej")) == abi.TRW_E_UNSUPPORTED
    assert ws(_params(abi, "node2vec", "naive")) == abi.TRW_E_UNSUPPORTED
    assert ws(_params(abi, "metapath", "alias")) == abi.TRW_E_UNSUPPORTED
    assert ws(_params(abi, "deepwalk", "naive", max_len=0)) == abi.TRW_E_INVALID
    assert ws(_params(abi, "deepwalk", "naive", max_len=65536)) == abi.TRW_E_INVALID
    assert ws(_params(abi, "node2vec", "orej", thr=(0, 1, 1))) == abi.TRW_E_INVALID
    assert ws(_params(abi, "node2vec", "orej", thr=(65537, 1, 1))) == abi.TRW_E_INVALID
    assert ws(_params(abi, "metapath", "its", schema=(1, 2))) == abi.TRW_E_INVALID   # no labels
    assert ws(_params(abi, "deepwalk", "naive"), nq=2**32) == abi.TRW_E_INVALID
    assert ws(_params(abi, "deepwalk", "naive"), mode=7) == abi.TRW_E_INVALID
    gl = _fake_graph(abi, labels=True)
    p = _params(abi, "metapath", "its", schema=())
    assert abi.trw_walk_workspace_bytes(gl, ctypes.byref(p), 1, 1, ctypes.byref(sz)) == abi.TRW_E_INVALID
    p = _params(abi, "metapath", "its", schema=(1, 2, 3))
    assert abi.trw_walk_workspace_bytes(gl, ctypes.byref(p), 1, 1, ctypes.byref(sz)) == abi.TRW_OK
    # per-step workspace grows with nq; persistent does not
    p = _params(abi, "ppr", "naive", max_len=256)
    abi.trw_walk_workspace_bytes(g, ctypes.byref(p), 1000, 0, ctypes.byref(sz))
    small = sz.value
    abi.trw_walk_workspace_bytes(g, ctypes.byref(p), 100000, 0, ctypes.byref(sz))
    assert sz.value > small
    abi.trw_walk_workspace_bytes(g, ctypes.byref(p), 100000, 1, ctypes.byref(sz))
    assert sz.value <= 256
    for h in (g, gl):
        abi.trw_graph_destroy(h)


def test_walk_argument_checks(abi):
    g = _fake_graph(abi, weights=True)
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x10000)
    def walk(p, table=None, stride=11, ws_ptr=ws, ws_bytes=1 << 20, nq=5):
        return abi.trw_walk(g, table, ctypes.byref(p), fake, nq, 0, fake, stride, fake, fake, 1, None,
                            ws_ptr, ws_bytes, None)
    assert walk(_params(abi, "deepwalk", "alias")) == abi.TRW_E_INVALID          # no table
    assert b"table" in abi.trw_last_error()
    assert walk(_params(abi, "ppr", "its")) == abi.TRW_E_INVALID
    assert walk(_params(abi, "deepwalk", "naive"), stride=10) == abi.TRW_E_INVALID
    assert walk(_params(abi, "deepwalk", "naive"), ws_ptr=ctypes.c_void_p(0x10010)) == abi.TRW_E_INVALID
    assert walk(_params(abi, "deepwalk", "naive"), ws_bytes=0) == abi.TRW_E_INVALID
    assert walk(_params(abi, "deepwalk", "naive"), nq=0) == abi.TRW_OK           # nothing to do
    sz = ctypes.c_size_t()
    assert abi.trw_table_bytes(g, abi.TRW_S_ALIAS, ctypes.byref(sz)) == abi.TRW_OK and sz.value == 32 * 1000
    assert abi.trw_table_bytes(g, abi.TRW_S_ITS, ctypes.byref(sz)) == abi.TRW_OK
    assert sz.value == 8192 + 32000 + 8 * 100      # prefix (256-aligned), slot records, W[n]
    assert abi.trw_table_bytes(g, abi.TRW_S_NAIVE, ctypes.byref(sz)) == abi.TRW_E_UNSUPPORTED
    t = ctypes.c_void_p()
    assert abi.trw_table_build(g, abi.TRW_S_ALIAS, fake, 10, None, ctypes.byref(t)) == abi.TRW_E_INVALID
    assert abi.trw_table_build(g, abi.TRW_S_ALIAS, ctypes.c_void_p(0x1010), 32000, None,
                               ctypes.byref(t)) == abi.TRW_E_INVALID
    # ITS: the search reads whole 64-byte prefix blocks, so the buffer must start on 256 bytes
    its_bytes = 8192 + 32000 + 8 * 100
    for misaligned in (0x1020, 0x1040, 0x1080):
        assert abi.trw_table_build(g, abi.TRW_S_ITS, ctypes.c_void_p(misaligned), its_bytes, None,
                                   ctypes.byref(t)) == abi.TRW_E_INVALID
        assert b"256-byte" in abi.trw_last_error()
    gn = _fake_graph(abi)
    assert abi.trw_table_build(gn, abi.TRW_S_ITS, fake, 8000, None, ctypes.byref(t)) == abi.TRW_E_INVALID
    abi.trw_graph_destroy(g)
    abi.trw_graph_destroy(gn)


def test_validate_sources_argument_checks(abi):
    """trw_validate_sources rejects bad arguments before any device work (none is done here)."""
    g = _fake_graph(abi)
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x10000)
    bad = ctypes.c_uint64(77)
    assert abi.trw_validate_sources(None, fake, 5, ws, 8, None, ctypes.byref(bad)) == abi.TRW_E_INVALID
    assert abi.trw_validate_sources(g, fake, 5, ws, 8, None, None) == abi.TRW_E_INVALID
    assert abi.trw_validate_sources(g, fake, 2**32, ws, 8, None, ctypes.byref(bad)) == abi.TRW_E_INVALID
    assert b"nq" in abi.trw_last_error()
    assert abi.trw_validate_sources(g, None, 5, ws, 8, None, ctypes.byref(bad)) == abi.TRW_E_INVALID
    assert abi.trw_validate_sources(g, fake, 5, None, 8, None, ctypes.byref(bad)) == abi.TRW_E_INVALID
    assert abi.trw_validate_sources(g, fake, 5, ws, 4, None, ctypes.byref(bad)) == abi.TRW_E_INVALID
    assert abi.trw_validate_sources(g, fake, 5, ctypes.c_void_p(0x10004), 8, None,
                                    ctypes.byref(bad)) == abi.TRW_E_INVALID
    assert bad.value == 77                           # untouched by a failing call
    abi.trw_graph_destroy(g)


def test_default_tuning(abi):
    from paper_2107_11983_amd import default_tuning
    g = _fake_graph(abi)
    t = abi.trw_tuning()
    p = _params(abi, "deepwalk", "naive")
    assert abi.trw_default_tuning(g, ctypes.byref(p), 1, ctypes.byref(t)) == abi.TRW_OK
    assert t.walkers_per_lane in (1, 2, 4) and t.block_threads % 64 == 0 and t.queue_chunk >= 1
    assert t.no_lds_graph == 0                       # small graphs walk from LDS unless told not to
    assert t.its_gallop_degree == 1                  # every ITS row searches from its guess
    assert t.n2v_search_degree == 0                  # Node2Vec always probes the edge index
    assert ctypes.sizeof(abi.trw_tuning) == 32       # the degree thresholds took the reserved words
    abi.trw_graph_destroy(g)


def test_rej_table_and_walk_checks(abi):
    g = _fake_graph(abi, weights=True)
    sz = ctypes.c_size_t()
    assert abi.trw_table_bytes(g, abi.TRW_S_REJ, ctypes.byref(sz)) == abi.TRW_OK
    assert sz.value == 32 * 1000 + 4 * 100          # 32 B per slot (already 256-aligned), then p*[n]
    fake = ctypes.c_void_p(0x1000)
    p = _params(abi, "ppr", "rej")
    assert abi.trw_walk(g, None, ctypes.byref(p), fake, 5, 0, fake, 11, fake, fake, 1, None,
                        ctypes.c_void_p(0x10000), 1 << 20, None) == abi.TRW_E_INVALID   # REJ needs its table
    assert _params(abi, "node2vec", "rej").sampler == abi.TRW_S_REJ
    assert abi.trw_walk_workspace_bytes(g, ctypes.byref(_params(abi, "node2vec", "rej")), 1, 1,
                                        ctypes.byref(sz)) == abi.TRW_E_UNSUPPORTED
    t = ctypes.c_void_p()
    gn = _fake_graph(abi)
    assert abi.trw_table_build(gn, abi.TRW_S_REJ, fake, 40000, None, ctypes.byref(t)) == abi.TRW_E_INVALID  # no w
    abi.trw_graph_destroy(g)
    abi.trw_graph_destroy(gn)


def test_ppr_estimate_argument_checks(abi):
    sz = ctypes.c_size_t()
    assert abi.trw_topk_workspace_bytes(100, 10, ctypes.byref(sz)) == abi.TRW_OK and sz.value == 1280 + 80
    assert abi.trw_topk_workspace_bytes(100, 101, ctypes.byref(sz)) == abi.TRW_E_INVALID
    assert abi.trw_topk_workspace_bytes(10**6, 4097, ctypes.byref(sz)) == abi.TRW_E_INVALID
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x10000)
    assert abi.trw_topk(fake, 100, 10, fake, fake, ws, 1000, None) == abi.TRW_E_INVALID          # short ws
    assert abi.trw_topk(fake, 100, 10, fake, fake, ctypes.c_void_p(0x10010), 4096, None) == abi.TRW_E_INVALID
    assert abi.trw_topk(None, 100, 10, fake, fake, ws, 4096, None) == abi.TRW_E_INVALID
    assert abi.trw_topk(fake, 2**31, 10, fake, fake, ws, 4096, None) == abi.TRW_E_INVALID
    assert abi.trw_topk(fake, 100, 0, None, None, None, 0, None) == abi.TRW_OK                   # k = 0
    g = _fake_graph(abi)                                                                        # n = 100
    def ec(nq, group, counts_len, stride=11, paths=fake):
        return abi.trw_ppr_end_counts(g, paths, stride, fake, fake, nq, group, fake, counts_len, None, None)
    assert ec(10, 0, 99) == abi.TRW_E_INVALID            # counts shorter than n
    assert ec(10, 3, 399) == abi.TRW_E_INVALID           # 4 groups of 3 need 400
    assert ec(10, 0, 100, stride=0) == abi.TRW_E_INVALID
    assert ec(10, 0, 100, paths=None) == abi.TRW_E_INVALID
    assert ec(2**32, 0, 100) == abi.TRW_E_INVALID
    assert ec(0, 0, 100) == abi.TRW_OK                   # nothing to do
    abi.trw_graph_destroy(g)


def test_ppr_walk_counts_argument_checks(abi):
    g = _fake_graph(abi, weights=True)                # n = 100
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x10000)
    def pc(p, counts=fake, counts_len=100, group=0, nq=5):
        return abi.trw_ppr_walk_counts(g, None, ctypes.byref(p), fake, nq, 0, group, counts, counts_len, fake,
                                       fake, None, ws, 1 << 20, None)
    assert pc(_params(abi, "deepwalk", "naive")) == abi.TRW_E_UNSUPPORTED
    assert pc(_params(abi, "ppr", "naive"), counts=None) == abi.TRW_E_INVALID
    assert pc(_params(abi, "ppr", "naive"), counts_len=99) == abi.TRW_E_INVALID
    assert pc(_params(abi, "ppr", "naive"), group=2, counts_len=200) == abi.TRW_E_INVALID   # 3 groups
    assert pc(_params(abi, "ppr", "alias")) == abi.TRW_E_INVALID                            # no table
    assert pc(_params(abi, "ppr", "naive"), nq=0) == abi.TRW_OK
    p = _params(abi, "ppr", "naive")                  # lengths and status: both or neither
    assert abi.trw_ppr_walk_counts(g, None, ctypes.byref(p), fake, 5, 0, 0, fake, 100, None, fake, None, ws,
                                   1 << 20, None) == abi.TRW_E_INVALID
    abi.trw_graph_destroy(g)


def test_walk_stream_argument_checks(abi):
    g = _fake_graph(abi)
    p = _params(abi, "ppr", "naive", max_len=10)
    dsz, hsz = ctypes.c_size_t(), ctypes.c_size_t()
    assert abi.trw_walk_stream_bytes(g, ctypes.byref(p), 0, ctypes.byref(dsz), ctypes.byref(hsz)) == abi.TRW_E_INVALID
    assert abi.trw_walk_stream_bytes(g, ctypes.byref(p), 100, ctypes.byref(dsz), ctypes.byref(hsz)) == abi.TRW_OK
    assert dsz.value > 2 * 100 * 16 * 4 and hsz.value > 2 * 100 * 11 * 4     # two chunk sets each
    fake = ctypes.c_void_p(0x1000)
    noop = abi.TRW_CHUNK_FN(lambda u, c: 0)
    def ws(d=ctypes.c_void_p(0x100000), db=None, h=ctypes.c_void_p(0x200000), hb=None, fn=noop, chunk=100):
        return abi.trw_walk_stream(g, None, ctypes.byref(p), fake, 5, 0, chunk, None, d,
                                   dsz.value if db is None else db, h, hsz.value if hb is None else hb,
                                   fn, None, None)
    assert ws(chunk=0) == abi.TRW_E_INVALID
    assert ws(db=100) == abi.TRW_E_INVALID
    assert ws(hb=100) == abi.TRW_E_INVALID
    assert ws(h=ctypes.c_void_p(0x200010)) == abi.TRW_E_INVALID
    assert ws(fn=abi.TRW_CHUNK_FN()) == abi.TRW_E_INVALID                     # NULL function
    abi.trw_graph_destroy(g)


def test_headers_are_plain_c(tmp_path):
    """include/*.h compile as strict C99 and as C++ (no C++ or torch types in the boundary)."""
    import subprocess
    src = tmp_path / "h.c"
    src.write_text('#include "trw.h"\n#include "trw_probe.h"\nint main(void) { return (int)trw_abi_version(); }\n')
    inc = os.path.join(ROOT, "include")
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                           "-I", inc, str(src)])
    subprocess.check_call(["g++", "-std=c++11", "-Wall", "-Werror", "-fsyntax-only", "-x", "c++", "-I", inc, str(src)])


def test_c_driver_builds(tmp_path):
    """The plain-C driver of the ABI compiles and links against libtrw.so with gcc."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("c_abi_build", os.path.join(ROOT, "tests", "c_abi", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    out = mod.build(str(tmp_path / "walk_from_c"))
    assert os.path.exists(out)


def test_placement_is_checked_before_any_device_call():
    """Graph and table placements other than device / host memory are refused in the binding."""
    import numpy as np
    import paper_2107_11983_amd as trw
    rp = np.array([0, 1, 1], np.int32)
    col = np.array([1], np.int32)
    with pytest.raises(ValueError):
        trw.Graph(rp, col, placement="disk")
    assert trw.PLACEMENTS == ("device", "host")


def test_label_index_sizes(abi):
    """Offsets, destinations, and for at most 6 labels the 32-byte fused entries (the documented layout)."""
    g = _fake_graph(abi, labels=True)               # n = 100, m = 1000
    r256 = lambda b: (b + 255) // 256 * 256
    b = ctypes.c_size_t(0)
    for L in (1, 5, 6):
        assert abi.trw_label_index_bytes(g, L, ctypes.byref(b)) == abi.TRW_OK
        assert b.value == r256(4 * 100 * (L + 1)) + r256(4 * 1000) + 32 * 1000, L
    for L in (7, 64):
        assert abi.trw_label_index_bytes(g, L, ctypes.byref(b)) == abi.TRW_OK
        assert b.value == r256(4 * 100 * (L + 1)) + 4 * 1000, L
    assert abi.trw_label_index_bytes(g, 65, ctypes.byref(b)) == abi.TRW_E_INVALID
    abi.trw_graph_destroy(g)


def test_walk_noalloc_size_limit(abi):
    """trw_walk_noalloc refuses a walk whose workspace exceeds its device array before any
    device work (the per-step schedule needs 32 bytes per query); nothing runs here."""
    g = _fake_graph(abi)
    fake = ctypes.c_void_p(0x1000)
    p = _params(abi, "deepwalk", "naive")
    limit = int(re.search(r"#define TRW_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", open(HEADER).read())
                .expand(r"\1")) << 20
    assert limit == 8 << 20
    nq = limit // 32 + 1
    st = abi.trw_walk_noalloc(g, None, ctypes.byref(p), fake, nq, 0, fake, 11, fake, fake, abi.TRW_M_PER_STEP,
                              None, None)
    assert st == abi.TRW_E_INVALID and b"workspace" in abi.trw_last_error()
    assert abi.trw_walk_noalloc(g, None, ctypes.byref(p), fake, 5, 0, fake, 11, fake, fake, 7, None,
                                None) == abi.TRW_E_INVALID         # unknown mode
    assert abi.trw_walk_noalloc(g, None, None, fake, 5, 0, fake, 11, fake, fake, 1, None,
                                None) == abi.TRW_E_INVALID         # no params
    abi.trw_graph_destroy(g)
