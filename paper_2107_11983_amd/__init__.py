"""MI355X random-walk engine: Python binding of libtrw.so.

PyTorch supplies device memory and streams; every step of the walk path runs
in the library's HIP kernels, reached through the C ABI (include/trw.h).
The binding marshals arguments and raises TrwError on any failing call.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

from . import _abi, programs  # noqa: F401  (programs: walk program sources)
from ._abi import (TRW_E_CANCELLED, TRW_E_INVALID, TRW_E_NOMEM_BUDGET, TRW_E_TIMEOUT, TRW_E_UNSUPPORTED,
                   TRW_REQ_HOST, trw_completion,
                   trw_request, trw_server_cfg, trw_server_stats)
from ._abi import (TRW_A_DEEPWALK, TRW_A_METAPATH, TRW_A_NODE2VEC, TRW_A_PPR, TRW_G_SYMMETRIC,
                   TRW_M_PER_STEP, TRW_M_PERSISTENT, TRW_S_ALIAS, TRW_S_ITS, TRW_S_NAIVE, TRW_S_OREJ, TRW_S_REJ,
                   TRW_ST_BAD_SOURCE, TRW_ST_DEAD_END, TRW_ST_LENGTH, TRW_ST_STOPPED, TrwError, check,
                   trw_tuning, trw_walk_params)

__all__ = ["Graph", "Table", "walk", "make_params", "workspace_bytes", "default_tuning", "autotune",
           "TrwError", "ALGOS", "SAMPLERS", "Program", "check_program", "programs", "Server", "ppr_end_counts",
           "ppr_walk_counts", "topk", "walk_stream", "walk_noalloc", "DiskGraph", "write_disk_graph"]

ALGOS = {"deepwalk": TRW_A_DEEPWALK, "ppr": TRW_A_PPR, "node2vec": TRW_A_NODE2VEC, "metapath": TRW_A_METAPATH}
SAMPLERS = {"naive": TRW_S_NAIVE, "alias": TRW_S_ALIAS, "its": TRW_S_ITS, "orej": TRW_S_OREJ, "rej": TRW_S_REJ}
MODES = {"per_step": TRW_M_PER_STEP, "persistent": TRW_M_PERSISTENT}


def _stream_ptr(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t: Optional[torch.Tensor]) -> Optional[ctypes.c_void_p]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _as_device(a, dtype_np, device) -> torch.Tensor:
    """numpy array -> device tensor with the same bits (uint32/uint8 kept bit-exact)."""
    if isinstance(a, torch.Tensor):
        return a.to(device)
    a = np.ascontiguousarray(a, dtype=dtype_np)
    if dtype_np == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(device)


def _as_pinned(a, dtype_np) -> torch.Tensor:
    """numpy array or tensor -> pinned host tensor with the same bits, which the device reads in place."""
    if isinstance(a, torch.Tensor):
        src = a.detach().to("cpu")
    else:
        a = np.ascontiguousarray(a, dtype=dtype_np)
        if dtype_np == np.uint32:
            a = a.view(np.int32)
        src = torch.from_numpy(a)
    out = torch.empty(src.shape, dtype=src.dtype, pin_memory=True)
    out.copy_(src)
    return out


PLACEMENTS = ("device", "host")


def stop_threshold(prob: float) -> int:
    """PPR stop coin threshold: a walk stops after a move iff r2 < floor(prob * 2^32)."""
    if not 0.0 <= prob <= 1.0:
        raise ValueError("stop probability must be in [0, 1]")
    return min(int(prob * 4294967296.0), 0xFFFFFFFF)


def n2v_thresholds(p: float, q: float) -> tuple:
    """Node2Vec dart thresholds in Q16: round(2^16 * p(e) / p*), clamped to [1, 65536].

    p(e) = 1/p for the previous vertex, 1 for its neighbours, 1/q otherwise
    (the Node2Vec transition equation); p* = max(1, 1/p, 1/q) is the O-REJ bound.
    """
    w = (1.0 / p, 1.0, 1.0 / q)
    top = max(w)
    return tuple(min(65536, max(1, int(round(65536.0 * x / top)))) for x in w)


def make_params(algo, sampler, max_len: int, seed: int, stop_q32: int = 0,
                n2v_thr_q16: Sequence[int] = (65536, 65536, 65536), schema: Sequence[int] = ()) -> trw_walk_params:
    """Fill trw_walk_params.  algo / sampler may be names ('ppr', 'alias') or enum values."""
    p = trw_walk_params()
    p.algo = ALGOS[algo] if isinstance(algo, str) else int(algo)
    p.sampler = SAMPLERS[sampler] if isinstance(sampler, str) else int(sampler)
    p.max_len = int(max_len)
    p.stop_q32 = int(stop_q32)
    for i in range(3):
        p.n2v_thr_q16[i] = int(n2v_thr_q16[i])
    p.schema_len = len(schema)
    for i, s in enumerate(schema):
        p.schema[i] = int(s)
    p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return p


class Graph:
    """A CSR graph wrapped in a trw_graph handle.

    row_ptr int32[n+1], col int32[m] (rows sorted, no duplicates), optional
    weight uint32[m] and label uint8[m].  The tensors live as long as the Graph.
    placement "device" copies them to the GPU; "host" keeps them in pinned host
    memory that the kernels read in place over the host link, for graphs larger
    than HBM (identical results, slower moves).  Tables follow the graph's
    placement unless told otherwise; walk outputs stay on the GPU.
    """

    def __init__(self, row_ptr, col, weight=None, label=None, symmetric: bool = False,
                 device: str = "cuda", placement: str = "device"):
        if placement not in PLACEMENTS:
            raise ValueError(f"placement must be one of {PLACEMENTS}")
        self.device = torch.device(device)
        self.placement = placement
        conv = ((lambda a, dt: _as_pinned(a, dt)) if placement == "host"
                else (lambda a, dt: _as_device(a, dt, self.device)))
        self.row_ptr = conv(row_ptr, np.int32)
        self.col = conv(col, np.int32)
        self.weight = None if weight is None else conv(weight, np.uint32)
        self.label = None if label is None else conv(label, np.uint8)
        self.n = self.row_ptr.numel() - 1
        self.m = self.col.numel()
        h = ctypes.c_void_p()
        check(_abi.trw_graph_create(self.n, self.m, _dptr(self.row_ptr), _dptr(self.col), _dptr(self.weight),
                                    _dptr(self.label), TRW_G_SYMMETRIC if symmetric else 0, ctypes.byref(h)))
        self.handle = h
        self._tables = []

    def validate(self, stream=None) -> int:
        ws = torch.empty(64, dtype=torch.uint8, device=self.device)
        bad = ctypes.c_uint64(0)
        st = _abi.trw_graph_validate(self.handle, _dptr(ws), 64, _stream_ptr(stream), ctypes.byref(bad))
        if st not in (0, _abi.TRW_E_INVALID):
            check(st)
        return int(bad.value)

    def validate_sources(self, sources: torch.Tensor, stream=None) -> int:
        """Number of sources outside [0, n) (trw_validate_sources; synchronises the stream)."""
        ws = torch.empty(8, dtype=torch.uint8, device=self.device)
        bad = ctypes.c_uint64(0)
        st = _abi.trw_validate_sources(self.handle, _dptr(sources), int(sources.numel()), _dptr(ws), 8,
                                       _stream_ptr(stream), ctypes.byref(bad))
        if st not in (0, _abi.TRW_E_INVALID) or (st != 0 and bad.value == 0):
            check(st)
        return int(bad.value)

    def table(self, sampler, stream=None, placement: Optional[str] = None) -> "Table":
        return Table(self, sampler, stream, placement=placement)

    def adjacency_index(self, stream=None, placement: Optional[str] = None) -> "Table":
        """Row-annotated adjacency for NAIVE / Node2Vec walks (identical results, fewer reads)."""
        return Table(self, "adjacency_index", stream, placement=placement)

    def edge_index(self, stream=None, placement: str = "device") -> "Table":
        """Adjacency index plus a hash set of the edges (Node2Vec's adjacency test in one probe).
        Built with device atomics, so in device memory whatever the graph's placement."""
        return Table(self, "edge_index", stream, placement=placement)

    def label_index(self, n_labels: int, stream=None, placement: Optional[str] = None) -> "Table":
        """MetaPath label index (rows sorted by label + per-vertex label offsets)."""
        return Table(self, "label_index", stream, n_labels=n_labels, placement=placement)

    def close(self):
        for t in list(self._tables):
            t.close()
        self._tables = []
        if self.handle:
            _abi.trw_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Table:
    """Per-vertex ALIAS, ITS or REJ table, or an index (built by the device, asynchronously,
    into device memory or, with placement "host", pinned host memory)."""

    def __init__(self, graph: Graph, sampler, stream=None, n_labels: int = 0, placement: Optional[str] = None):
        self.graph = graph
        self.placement = placement or graph.placement
        if self.placement not in PLACEMENTS:
            raise ValueError(f"placement must be one of {PLACEMENTS}")
        nbytes = ctypes.c_size_t(0)
        h = ctypes.c_void_p()

        def buf(nb: int) -> torch.Tensor:
            if self.placement == "host":
                self._keep, t = _aligned(nb, pin=True)
                return t
            return torch.empty(nb, dtype=torch.uint8, device=graph.device)

        if sampler == "adjacency_index":
            self.sampler = None
            check(_abi.trw_adjacency_index_bytes(graph.handle, ctypes.byref(nbytes)))
            self.buf = buf(max(int(nbytes.value), 16))
            check(_abi.trw_adjacency_index_build(graph.handle, _dptr(self.buf), int(nbytes.value),
                                                 _stream_ptr(stream), ctypes.byref(h)))
        elif sampler == "edge_index":
            self.sampler = None
            check(_abi.trw_edge_index_bytes(graph.handle, ctypes.byref(nbytes)))
            self.buf = buf(int(nbytes.value))
            check(_abi.trw_edge_index_build(graph.handle, _dptr(self.buf), int(nbytes.value),
                                            _stream_ptr(stream), ctypes.byref(h)))
        elif sampler == "label_index":
            self.sampler = None
            self.n_labels = n_labels
            check(_abi.trw_label_index_bytes(graph.handle, n_labels, ctypes.byref(nbytes)))
            self.buf = buf(max(int(nbytes.value), 256))
            check(_abi.trw_label_index_build(graph.handle, n_labels, _dptr(self.buf), int(nbytes.value),
                                             _stream_ptr(stream), ctypes.byref(h)))
        else:
            self.sampler = SAMPLERS[sampler] if isinstance(sampler, str) else int(sampler)
            check(_abi.trw_table_bytes(graph.handle, self.sampler, ctypes.byref(nbytes)))
            self.buf = buf(max(int(nbytes.value), 16))
            check(_abi.trw_table_build(graph.handle, self.sampler, _dptr(self.buf), int(nbytes.value),
                                       _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        graph._tables.append(self)

    def close(self):
        """Destroy the handle and release the table's memory (the graph forgets it too)."""
        if self.handle:
            _abi.trw_table_destroy(self.handle)
            self.handle = None
        self.buf = None
        self._keep = None
        if self in self.graph._tables:
            self.graph._tables.remove(self)


def workspace_bytes(graph: Graph, p: trw_walk_params, nq: int, mode=TRW_M_PERSISTENT) -> int:
    out = ctypes.c_size_t(0)
    check(_abi.trw_walk_workspace_bytes(graph.handle, ctypes.byref(p), nq, MODES.get(mode, mode), ctypes.byref(out)))
    return int(out.value)


def default_tuning(graph: Graph, p: trw_walk_params, mode=TRW_M_PERSISTENT) -> trw_tuning:
    t = trw_tuning()
    check(_abi.trw_default_tuning(graph.handle, ctypes.byref(p), MODES.get(mode, mode), ctypes.byref(t)))
    return t


def make_tuning(**kw) -> trw_tuning:
    t = trw_tuning()
    for k, v in kw.items():
        setattr(t, k, int(v))
    return t


class WalkBuffers:
    """Output and scratch buffers for repeated walks of the same shape."""

    def __init__(self, graph: Graph, p: trw_walk_params, nq: int, mode=TRW_M_PERSISTENT, stride: int = 0):
        self.nq = nq
        # 64-byte rows: a path's last block is then written whole (entries past a path's end are unspecified)
        self.stride = stride or ((p.max_len + 1 + 15) // 16 * 16)
        dev = graph.device
        self.paths = torch.empty((nq, self.stride), dtype=torch.int32, device=dev)
        self.lengths = torch.empty(nq, dtype=torch.int32, device=dev)
        self.status = torch.empty(nq, dtype=torch.uint8, device=dev)
        self.ws = torch.empty(max(workspace_bytes(graph, p, nq, mode), 256), dtype=torch.uint8, device=dev)


def walk(graph: Graph, table: Optional[Table], p: trw_walk_params, sources: torch.Tensor, qid_base: int = 0,
         mode=TRW_M_PERSISTENT, tuning: Optional[trw_tuning] = None, bufs: Optional[WalkBuffers] = None,
         stream=None):
    """Run len(sources) queries; returns (paths int32[nq, stride], lengths, status).

    lengths are uint32 values held in an int32 tensor (moves per query, <= 65535).
    """
    mode = MODES.get(mode, mode)
    nq = int(sources.numel())
    if bufs is None:
        bufs = WalkBuffers(graph, p, nq, mode)
    assert bufs.nq == nq
    check(_abi.trw_walk(graph.handle, table.handle if table is not None else None, ctypes.byref(p),
                        _dptr(sources), nq, qid_base, _dptr(bufs.paths), bufs.stride, _dptr(bufs.lengths),
                        _dptr(bufs.status), mode, ctypes.byref(tuning) if tuning is not None else None,
                        _dptr(bufs.ws), bufs.ws.numel(), _stream_ptr(stream)))
    return bufs.paths, bufs.lengths, bufs.status


def walk_noalloc(graph: Graph, table: Optional[Table], p: trw_walk_params, sources: torch.Tensor,
                 paths: torch.Tensor, lengths: torch.Tensor, status: torch.Tensor, qid_base: int = 0,
                 mode=TRW_M_PERSISTENT, tuning: Optional[trw_tuning] = None, stream=None):
    """trw_walk_noalloc: the walk with the library's own device workspace (no allocation in the
    call); the caller passes the outputs (paths int32[nq, stride], lengths, status)."""
    mode = MODES.get(mode, mode)
    nq = int(sources.numel())
    check(_abi.trw_walk_noalloc(graph.handle, table.handle if table is not None else None, ctypes.byref(p),
                                _dptr(sources), nq, qid_base, _dptr(paths), paths.stride(0), _dptr(lengths),
                                _dptr(status), mode, ctypes.byref(tuning) if tuning is not None else None,
                                _stream_ptr(stream)))
    return paths, lengths, status


def autotune(graph: Graph, table: Optional[Table], p: trw_walk_params, sources: torch.Tensor,
             mode=TRW_M_PERSISTENT, budget: int = 0, stream=None):
    """Pre-execute walks under candidate tunings; returns (best trw_tuning, best ms)."""
    mode = MODES.get(mode, mode)
    nq = int(sources.numel())
    bufs = WalkBuffers(graph, p, nq, mode)
    out = trw_tuning()
    ms = ctypes.c_float(0)
    check(_abi.trw_autotune(graph.handle, table.handle if table is not None else None, ctypes.byref(p),
                            _dptr(sources), nq, _dptr(bufs.paths), bufs.stride, _dptr(bufs.lengths),
                            _dptr(bufs.status), mode, budget, _dptr(bufs.ws), bufs.ws.numel(),
                            _stream_ptr(stream), ctypes.byref(out), ctypes.byref(ms)))
    return out, float(ms.value)


def ppr_end_counts(graph: Graph, paths: torch.Tensor, lengths: torch.Tensor, status: torch.Tensor, group: int = 0,
                   counts: Optional[torch.Tensor] = None, skipped: Optional[torch.Tensor] = None, stream=None):
    """PPR estimate: add each query's end vertex to counts[query // group] (group 0: one row).

    Returns counts (uint32 values in an int32 tensor [groups, n], added to when given) and
    skipped (a one-element int64 tensor: bad sources and paths whose end is not a vertex).
    """
    nq = int(lengths.numel())
    stride = int(paths.shape[1]) if paths.dim() == 2 else int(paths.stride(0))
    groups = 1 if group <= 0 else max(1, -(-nq // group))
    if counts is None:
        counts = torch.zeros((groups, graph.n), dtype=torch.int32, device=graph.device)
    if skipped is None:
        skipped = torch.zeros(1, dtype=torch.int64, device=graph.device)
    assert counts.dtype == torch.int32 and counts.is_contiguous() and skipped.dtype == torch.int64
    assert paths.is_contiguous() or paths.stride(1) == 1
    check(_abi.trw_ppr_end_counts(graph.handle, _dptr(paths), paths.stride(0), _dptr(lengths), _dptr(status), nq,
                                  max(group, 0), _dptr(counts), counts.numel(), _dptr(skipped), _stream_ptr(stream)))
    return counts, skipped


def ppr_walk_counts(graph: Graph, table: Optional[Table], p: trw_walk_params, sources: torch.Tensor, group: int = 0,
                    qid_base: int = 0, counts: Optional[torch.Tensor] = None, tuning: Optional[trw_tuning] = None,
                    outputs: bool = True, stream=None):
    """PPR walks that count their end vertices instead of writing paths.

    Returns (counts [groups, n] as in ppr_end_counts, lengths, status); counts are added to when given.
    With outputs=False nothing is stored per query and lengths and status are None.
    """
    nq = int(sources.numel())
    groups = 1 if group <= 0 else max(1, -(-nq // group))
    if counts is None:
        counts = torch.zeros((groups, graph.n), dtype=torch.int32, device=graph.device)
    lengths = torch.empty(max(nq, 1), dtype=torch.int32, device=graph.device) if outputs else None
    status = torch.empty(max(nq, 1), dtype=torch.uint8, device=graph.device) if outputs else None
    ws = torch.empty(max(workspace_bytes(graph, p, nq, TRW_M_PERSISTENT), 256), dtype=torch.uint8,
                     device=graph.device)
    check(_abi.trw_ppr_walk_counts(graph.handle, table.handle if table is not None else None, ctypes.byref(p),
                                   _dptr(sources), nq, qid_base, max(group, 0), _dptr(counts), counts.numel(),
                                   _dptr(lengths) if outputs else None, _dptr(status) if outputs else None,
                                   ctypes.byref(tuning) if tuning is not None else None,
                                   _dptr(ws), ws.numel(), _stream_ptr(stream)))
    if not outputs:
        return counts, None, None
    return counts, lengths[:nq], status[:nq]


def _aligned(nbytes: int, device=None, pin: bool = False):
    """A uint8 tensor of at least nbytes whose storage starts on 256 bytes (and the tensor kept alive)."""
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=device, pin_memory=pin)
    off = (-t.data_ptr()) % 256
    return t, t[off:off + nbytes]


def _stream_buffers(graph: Graph, p: trw_walk_params, chunk_queries: int):
    dbytes, hbytes = ctypes.c_size_t(0), ctypes.c_size_t(0)
    check(_abi.trw_walk_stream_bytes(graph.handle, ctypes.byref(p), chunk_queries, ctypes.byref(dbytes),
                                     ctypes.byref(hbytes)))
    d_keep, d_ws = _aligned(int(dbytes.value), device=graph.device)
    h_keep, h_buf = _aligned(int(hbytes.value), pin=True)
    return d_keep, d_ws, h_keep, h_buf


def walk_stream(graph: Graph, table: Optional[Table], p: trw_walk_params, sources: torch.Tensor, chunk_queries: int,
                fn, qid_base: int = 0, tuning: Optional[trw_tuning] = None, stream=None) -> int:
    """Streamed walk (trw_walk_stream): the batch runs chunk_queries at a time and fn(chunk) is
    called on this thread for each chunk, in order, while the next chunk walks.  chunk is a dict
    with qid_base, nq and numpy copies of lengths, status, offsets (nq + 1) and entries (the
    packed paths: query i's path is entries[offsets[i]:offsets[i + 1]]).  fn returning True stops
    the stream (TrwError TRW_E_CANCELLED).  Returns the number of chunks delivered."""
    nq = int(sources.numel())
    d_keep, d_ws, h_keep, h_buf = _stream_buffers(graph, p, chunk_queries)
    delivered = [0]
    err = []

    def _cb(_user, cp):
        try:
            c = cp.contents
            n = int(c.nq)
            offs = np.ctypeslib.as_array(ctypes.cast(c.offsets, ctypes.POINTER(ctypes.c_uint64)), (n + 1,)).copy()
            total = int(offs[n])
            ent = (np.ctypeslib.as_array(ctypes.cast(c.entries, ctypes.POINTER(ctypes.c_int32)), (total,)).copy()
                   if total else np.zeros(0, np.int32))
            chunk = {"qid_base": int(c.qid_base), "nq": n,
                     "lengths": np.ctypeslib.as_array(ctypes.cast(c.lengths, ctypes.POINTER(ctypes.c_uint32)),
                                                      (n,)).copy(),
                     "status": np.ctypeslib.as_array(ctypes.cast(c.status, ctypes.POINTER(ctypes.c_uint8)),
                                                     (n,)).copy(),
                     "offsets": offs, "entries": ent}
            delivered[0] += 1
            return 1 if fn(chunk) else 0
        except Exception as e:   # surface the callback's error after the call
            err.append(e)
            return 1

    cb = _abi.TRW_CHUNK_FN(_cb)
    st = _abi.trw_walk_stream(graph.handle, table.handle if table is not None else None, ctypes.byref(p),
                              _dptr(sources), nq, qid_base, chunk_queries,
                              ctypes.byref(tuning) if tuning is not None else None, _dptr(d_ws), d_ws.numel(),
                              ctypes.c_void_p(h_buf.data_ptr()), h_buf.numel(), cb, None, _stream_ptr(stream))
    del d_keep, h_keep
    if err:
        raise err[0]
    check(st)
    return delivered[0]


def walk_stream_to_file(graph: Graph, table: Optional[Table], p: trw_walk_params, sources: torch.Tensor,
                        chunk_queries: int, path: str, qid_base: int = 0, tuning: Optional[trw_tuning] = None,
                        stream=None) -> int:
    """Streamed walk whose chunks the library itself appends to the file at `path`
    (trw_chunk_to_fd: the disk write of one chunk overlaps the walk of the next).  The file is
    created or truncated; read it back with read_stream_file.  Returns the bytes written."""
    nq = int(sources.numel())
    d_keep, d_ws, h_keep, h_buf = _stream_buffers(graph, p, chunk_queries)
    fd = os.open(path, os.O_WRONLY | os.O_CREAT | os.O_TRUNC, 0o644)
    try:
        fd_box = ctypes.c_int(fd)
        st = _abi.trw_walk_stream(graph.handle, table.handle if table is not None else None, ctypes.byref(p),
                                  _dptr(sources), nq, qid_base, chunk_queries,
                                  ctypes.byref(tuning) if tuning is not None else None, _dptr(d_ws), d_ws.numel(),
                                  ctypes.c_void_p(h_buf.data_ptr()), h_buf.numel(), _abi.TRW_CHUNK_TO_FD,
                                  ctypes.byref(fd_box), _stream_ptr(stream))
    finally:
        os.close(fd)
    del d_keep, h_keep
    check(st)
    return os.path.getsize(path)


def read_stream_file(path: str):
    """The chunks of a file written by walk_stream_to_file, in order, as the dicts walk_stream
    hands to its function."""
    data = np.fromfile(path, dtype=np.uint8)
    pos = 0
    while pos < data.size:
        qid_base = int(data[pos:pos + 8].view(np.uint64)[0])
        n = int(data[pos + 8:pos + 12].view(np.uint32)[0])
        pos += 16
        lengths = data[pos:pos + 4 * n].view(np.uint32).copy()
        pos += 4 * n
        status = data[pos:pos + n].copy()
        pos += n + (8 - n % 8) % 8
        offs = data[pos:pos + 8 * (n + 1)].view(np.uint64).copy()
        pos += 8 * (n + 1)
        total = int(offs[n])
        entries = data[pos:pos + 4 * total].view(np.int32).copy()
        pos += 4 * total
        yield {"qid_base": qid_base, "nq": n, "lengths": lengths, "status": status, "offsets": offs,
               "entries": entries}


def write_disk_graph(path: str, row_ptr, col, weight=None, label=None) -> None:
    """Write a CSR file for DiskGraph (trw_disk_graph_write) from host arrays: row_ptr as
    int64[n + 1], col int32[m], optional weight uint32[m] and label uint8[m]."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    w = None if weight is None else np.ascontiguousarray(weight, dtype=np.uint32)
    lab = None if label is None else np.ascontiguousarray(label, dtype=np.uint8)
    n, m = rp.size - 1, c.size
    check(_abi.trw_disk_graph_write(path.encode(), n, m, rp.ctypes.data, c.ctypes.data if m else None,
                                    None if w is None else w.ctypes.data, None if lab is None else lab.ctypes.data))


class DiskGraph:
    """A CSR graph kept in a file (trw_disk_graph_*): walks load one vertex-range partition
    of at most part_edges edges onto the device at a time."""

    def __init__(self, path: str, part_edges: int = 0):
        h = ctypes.c_void_p()
        check(_abi.trw_disk_graph_open(path.encode(), part_edges, ctypes.byref(h)))
        self.handle = h
        n, m = ctypes.c_uint64(0), ctypes.c_uint64(0)
        flags, parts = ctypes.c_uint32(0), ctypes.c_uint32(0)
        check(_abi.trw_disk_graph_info(h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(flags), ctypes.byref(parts)))
        self.n, self.m, self.flags, self.parts = int(n.value), int(m.value), int(flags.value), int(parts.value)

    def partition(self, i: int):
        """(v_begin, v_end, e_begin, e_end) of partition i."""
        vals = [ctypes.c_int64(0) for _ in range(4)]
        check(_abi.trw_disk_graph_partition(self.handle, i, *[ctypes.byref(v) for v in vals]))
        return tuple(int(v.value) for v in vals)

    def walk_bytes(self, p: trw_walk_params, nq: int, slots: int = 1):
        d, h = ctypes.c_size_t(0), ctypes.c_size_t(0)
        check(_abi.trw_disk_walk_bytes(self.handle, ctypes.byref(p), nq, slots, ctypes.byref(d), ctypes.byref(h)))
        return int(d.value), int(h.value)

    def walk(self, p: trw_walk_params, sources: torch.Tensor, qid_base: int = 0, stride: Optional[int] = None,
             slots: int = 1, stream=None):
        """Run len(sources) queries (device int32 sources) with up to `slots` partitions resident;
        returns (paths int32[nq, stride], lengths, status, stats dict), the outputs those of
        trw_walk on the whole graph."""
        nq = int(sources.numel())
        dev = sources.device
        stride = stride or int(p.max_len) + 1
        paths = torch.empty((nq, stride), dtype=torch.int32, device=dev)
        lengths = torch.empty(nq, dtype=torch.int32, device=dev)
        status = torch.empty(nq, dtype=torch.uint8, device=dev)
        dbytes, hbytes = self.walk_bytes(p, nq, slots) if nq else (0, 0)
        d_keep, d_ws = _aligned(max(dbytes, 256), device=dev)
        h_keep, h_buf = _aligned(max(hbytes, 256), pin=True)
        stats = _abi.trw_disk_walk_stats()
        check(_abi.trw_disk_walk(self.handle, ctypes.byref(p), _dptr(sources), nq, qid_base, _dptr(paths), stride,
                                 _dptr(lengths), _dptr(status), slots, _dptr(d_ws), d_ws.numel(),
                                 ctypes.c_void_p(h_buf.data_ptr()), h_buf.numel(), ctypes.byref(stats),
                                 _stream_ptr(stream)))
        del d_keep, h_keep
        return paths, lengths, status, stats.as_dict()

    def close(self):
        if self.handle:
            check(_abi.trw_disk_graph_close(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def topk(counts: torch.Tensor, k: int, stream=None):
    """The k largest counts of a 1-D uint32 (int32-held) tensor: (ids int32[k], counts int32[k]),
    largest first, equal counts by the smaller index."""
    assert counts.dim() == 1 and counts.is_contiguous() and counts.dtype == torch.int32
    n = int(counts.numel())
    nbytes = ctypes.c_size_t(0)
    check(_abi.trw_topk_workspace_bytes(n, k, ctypes.byref(nbytes)))
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=counts.device)
    ids = torch.empty(max(k, 1), dtype=torch.int32, device=counts.device)
    vals = torch.empty(max(k, 1), dtype=torch.int32, device=counts.device)
    check(_abi.trw_topk(_dptr(counts), n, k, _dptr(ids), _dptr(vals), _dptr(ws), ws.numel(), _stream_ptr(stream)))
    return ids[:k], vals[:k]


class Server:
    """Continuous-batching walk server (C ABI trw_server_*): the graph and tables stay
    resident; requests of different sizes are admitted as memory frees up and share the
    device tick by tick.  Outputs are device tensors allocated here (or host arrays with
    host=True) and stay referenced until their completion is polled."""

    def __init__(self, graph: Graph, alias: Optional[Table] = None, adjacency: Optional[Table] = None,
                 pool_bytes: int = 1 << 30, max_slots: int = 0, max_requests: int = 0, steps_per_tick: int = 0,
                 use_hipgraph: bool = True, pipelined: bool = True, ring_chunks: int = 0):
        self.graph = graph
        cfg = trw_server_cfg()
        cfg.max_slots, cfg.max_requests, cfg.steps_per_tick = max_slots, max_requests, steps_per_tick
        cfg.use_hipgraph = 1 if use_hipgraph else 0
        cfg.serial_ticks = 0 if pipelined else 1
        cfg.ring_chunks = ring_chunks
        nbytes = ctypes.c_size_t(0)
        check(_abi.trw_server_arena_bytes(ctypes.byref(cfg), pool_bytes, ctypes.byref(nbytes)))
        self.arena = torch.empty(int(nbytes.value), dtype=torch.uint8, device=graph.device)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        check(_abi.trw_server_create(graph.handle, alias.handle if alias else None,
                                     adjacency.handle if adjacency else None, ctypes.byref(cfg),
                                     _dptr(self.arena), int(nbytes.value), ctypes.byref(h)))
        self.handle = h
        self._live = {}

    def submit(self, p: trw_walk_params, sources, qid_base: int = 0, host: bool = False, stride: int = 0) -> int:
        """Queue len(sources) queries; returns the request id."""
        nq = len(sources)
        stride = stride or ((p.max_len + 1 + 7) // 8 * 8)
        r = trw_request()
        r.params = p
        r.nq = nq
        r.qid_base = qid_base
        r.path_stride = stride
        if host:
            src = np.ascontiguousarray(sources, dtype=np.int32)
            out = (np.empty((nq, stride), np.int32), np.empty(nq, np.uint32), np.empty(nq, np.uint8))
            ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
            r.flags = TRW_REQ_HOST
        else:
            src = sources if isinstance(sources, torch.Tensor) else torch.from_numpy(
                np.ascontiguousarray(sources, dtype=np.int32)).to(self.graph.device)
            out = (torch.empty((nq, stride), dtype=torch.int32, device=self.graph.device),
                   torch.empty(nq, dtype=torch.int32, device=self.graph.device),
                   torch.empty(nq, dtype=torch.uint8, device=self.graph.device))
            ptr = lambda a: ctypes.c_void_p(a.data_ptr())
            torch.cuda.current_stream().synchronize()      # sources / outputs ready before the server's stream reads them
        r.sources = ptr(src)
        r.paths, r.lengths, r.status = ptr(out[0]), ptr(out[1]), ptr(out[2])
        rid = ctypes.c_uint64(0)
        check(_abi.trw_server_submit(self.handle, ctypes.byref(r), ctypes.byref(rid)))
        self._live[int(rid.value)] = (src, out)
        return int(rid.value)

    def cancel(self, request_id: int) -> None:
        check(_abi.trw_server_cancel(self.handle, request_id))

    def poll(self, max_n: int = 256, timeout_ms: int = 0):
        """Completed requests: list of dicts with request_id, status, times and the outputs."""
        buf = (trw_completion * max_n)()
        n = ctypes.c_uint32(0)
        st = _abi.trw_server_poll(self.handle, buf, max_n, ctypes.byref(n), timeout_ms)
        if st not in (0, TRW_E_TIMEOUT):
            check(st)
        res = []
        for i in range(n.value):
            c = buf[i]
            src, out = self._live.pop(int(c.request_id))
            res.append(dict(request_id=int(c.request_id), status=int(c.status), nq=int(c.nq),
                            t_submit_ns=int(c.t_submit_ns), t_admit_ns=int(c.t_admit_ns), t_done_ns=int(c.t_done_ns),
                            paths=out[0], lengths=out[1], status_codes=out[2]))
        return res

    def stats(self) -> dict:
        st = trw_server_stats()
        check(_abi.trw_server_stats_get(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self.handle:
            _abi.trw_server_destroy(self.handle)
            self.handle = None
            self._live = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Walk programs (C ABI trw_program_*): user-written sampling rules compiled at
# run time against csrc/program_rt.hpp.
# ---------------------------------------------------------------------------
PROGRAM_KINDS = {"static_naive": 0, "static_alias": 1, "static_its": 2, "dynamic_rej": 3, "dynamic_its": 4,
                 "static_rej": 5}


def check_program(source: str, arch: str = "gfx950") -> None:
    """Compile a walk program without loading it (no GPU needed); raises TrwError with the log."""
    check(_abi.trw_program_check(source.encode(), arch.encode()))


class Program:
    """A walk program: `struct TrwProgram` (kind, weight, update) in HIP C++."""

    def __init__(self, source: str):
        h = ctypes.c_void_p()
        check(_abi.trw_program_create(source.encode(), ctypes.byref(h)))
        self.handle = h
        k = ctypes.c_uint32(0)
        check(_abi.trw_program_kind(h, ctypes.byref(k)))
        self.kind = int(k.value)

    def walk(self, graph: Graph, table: Optional[Table], sources: torch.Tensor, max_len: int, seed: int,
             user: Sequence[int] = (), qid_base: int = 0, stride: int = 0, stream=None):
        """Run len(sources) queries; returns (paths int32[nq, stride], lengths, status) like walk()."""
        nq = int(sources.numel())
        pp = _abi.trw_program_params()
        pp.max_len = int(max_len)
        pp.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        for i, v in enumerate(user):
            pp.user[i] = int(v) & 0xFFFFFFFF
        stride = stride or ((max_len + 1 + 15) // 16 * 16)
        dev = graph.device
        paths = torch.empty((nq, stride), dtype=torch.int32, device=dev)
        lengths = torch.empty(nq, dtype=torch.int32, device=dev)
        status = torch.empty(nq, dtype=torch.uint8, device=dev)
        ws = torch.empty(256, dtype=torch.uint8, device=dev)
        check(_abi.trw_program_walk(self.handle, graph.handle, table.handle if table is not None else None,
                                    ctypes.byref(pp), _dptr(sources), nq, qid_base, _dptr(paths), stride,
                                    _dptr(lengths), _dptr(status), _dptr(ws), ws.numel(), _stream_ptr(stream)))
        self._ws = ws
        return paths, lengths, status

    def close(self):
        if self.handle:
            _abi.trw_program_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
