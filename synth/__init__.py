"""Seeded synthetic inputs shared by the oracle and the HIP path.

Only inputs live here: R-MAT graphs in CSR form, edge weights and labels,
query sources, MetaPath schemas and serving arrival traces.  None of the
random-walk method's arithmetic is in this module.  The native part is
``rmat.c`` (built with gcc into ``librmat.so``).

The paper evaluates on real graphs with weights drawn uniformly from a range
and five uniform edge labels (Experimental Setup, "Workloads"); the workloads
below are R-MAT stand-ins with the same structure (power-law degrees,
uniform weights and labels), at the sizes named in ``WORKLOADS``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmat.c")
_LIB = os.path.join(_HERE, "librmat.so")
_lib = None

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = True) -> str:
    """Compile rmat.c into librmat.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.synth_rmat_csr.restype = ctypes.c_int64
        lib.synth_rmat_csr.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_uint64, P, P]
        lib.synth_edge_attrs.restype = ctypes.c_int
        lib.synth_edge_attrs.argtypes = [ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, P, P]
        lib.synth_sources.restype = ctypes.c_int
        lib.synth_sources.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, P]
        lib.synth_uniform_u32.restype = ctypes.c_int
        lib.synth_uniform_u32.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, P]
        lib.synth_uniform_f64.restype = ctypes.c_int
        lib.synth_uniform_f64.argtypes = [ctypes.c_int64, ctypes.c_uint64, P]
        lib.synth_permutation.restype = ctypes.c_int
        lib.synth_permutation.argtypes = [ctypes.c_int64, ctypes.c_uint64, P]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


@dataclass
class CSRGraph:
    """Host CSR graph: rows sorted ascending, no self-loops, no duplicates."""
    n: int
    row_ptr: np.ndarray            # int32[n+1]
    col: np.ndarray                # int32[m]
    weight: Optional[np.ndarray] = None   # uint32[m]
    label: Optional[np.ndarray] = None    # uint8[m]
    symmetric: bool = False
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def rmat(scale: int, avg_degree: float, symmetric: bool, seed: int,
         abc=RMAT_ABC) -> CSRGraph:
    """R-MAT graph with n = 2^scale vertices.

    Directed graphs draw n*avg_degree samples; symmetric graphs draw
    n*avg_degree/2 samples and emit both directions.  Self-loops and duplicate
    edges are removed, so the realized m is below the nominal n*avg_degree.
    """
    lib = _load()
    n = 1 << scale
    nominal = int(round(n * avg_degree))
    n_samples = nominal // 2 if symmetric else nominal
    cap = n_samples * (2 if symmetric else 1)
    row_ptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(max(cap, 1), dtype=np.int32)
    m = lib.synth_rmat_csr(scale, n_samples, abc[0], abc[1], abc[2], 1 if symmetric else 0,
                           seed & 0xFFFFFFFFFFFFFFFF, _ptr(row_ptr), _ptr(col))
    if m < 0:
        raise MemoryError("synth_rmat_csr: allocation failed")
    if m >= 2 ** 31:
        raise ValueError("graph has >= 2^31 edges; int32 CSR cannot hold it")
    col = col[:m].copy() if m < cap // 2 else col[:m]
    g = CSRGraph(n=n, row_ptr=row_ptr.astype(np.int32), col=col, symmetric=symmetric,
                 meta=dict(scale=scale, avg_degree=avg_degree, seed=seed, abc=tuple(abc),
                           samples=n_samples))
    return g


def attach_attrs(g: CSRGraph, seed: int, weights: bool = False, labels: int = 0,
                 w_range=(1, 255)) -> CSRGraph:
    """Attach uint32 weights uniform in w_range and/or uint8 labels uniform in [0, labels)."""
    lib = _load()
    rp64 = g.row_ptr.astype(np.int64)
    w = np.empty(g.m, dtype=np.uint32) if weights else None
    lab = np.empty(g.m, dtype=np.uint8) if labels else None
    lib.synth_edge_attrs(g.n, _ptr(rp64), _ptr(g.col), 1 if g.symmetric else 0,
                         seed & 0xFFFFFFFFFFFFFFFF, w_range[0], w_range[1], max(labels, 1),
                         _ptr(w), _ptr(lab))
    g.weight = w
    g.label = lab
    return g


def sources(nq: int, n: int, seed: int) -> np.ndarray:
    """nq query sources drawn uniformly from [0, n)."""
    out = np.empty(nq, dtype=np.int32)
    _load().synth_sources(nq, n, seed & 0xFFFFFFFFFFFFFFFF, _ptr(out))
    return out


def uniform_u32(count: int, bound: int, seed: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint32)
    _load().synth_uniform_u32(count, bound, seed & 0xFFFFFFFFFFFFFFFF, _ptr(out))
    return out


def uniform_f64(count: int, seed: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().synth_uniform_f64(count, seed & 0xFFFFFFFFFFFFFFFF, _ptr(out))
    return out


def from_edges(n: int, edges, weights=None, labels=None) -> CSRGraph:
    """Small hand-written graphs for tests: list of (u, v) directed edges."""
    edges = list(edges)
    order = sorted(range(len(edges)), key=lambda i: (edges[i][0], edges[i][1]))
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    col = np.empty(len(edges), dtype=np.int32)
    for pos, i in enumerate(order):
        u, v = edges[i]
        row_ptr[u + 1] += 1
        col[pos] = v
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    g = CSRGraph(n=n, row_ptr=row_ptr, col=col)
    if weights is not None:
        g.weight = np.array([weights[i] for i in order], dtype=np.uint32)
    if labels is not None:
        g.label = np.array([labels[i] for i in order], dtype=np.uint8)
    return g


# ---------------------------------------------------------------------------
# Workloads.  Each is an R-MAT stand-in for one of the paper's workload shapes
# (Experimental Setup; Scalability Evaluation).  Seeds are fixed so that every
# run, on any machine, sees the same graph, sources and schema.
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    scale: int
    avg_degree: float
    symmetric: bool
    weights: bool
    labels: int
    algo: str              # deepwalk | ppr | node2vec | metapath | mixed
    samplers: tuple
    max_len: int
    nq: Optional[int]      # None: one query per vertex
    graph_seed: int
    walk_seed: int
    src_seed: int
    stop_prob: float = 0.0
    n2v_pq: tuple = (2.0, 0.5)
    schema_len: int = 0


WORKLOADS = {
    "deepwalk-rmat12": Workload("deepwalk-rmat12", 12, 16, True, False, 0, "deepwalk", ("naive",),
                                80, None, 0x7452570001, 0x5EED000001, 0x5AC0000001),
    "ppr-rmat22": Workload("ppr-rmat22", 22, 32, False, True, 0, "ppr", ("alias", "its"),
                           256, 10_000_000, 0x7452570002, 0x5EED000002, 0x5AC0000002, stop_prob=0.2),
    "node2vec-rmat24": Workload("node2vec-rmat24", 24, 16, True, False, 0, "node2vec", ("orej",),
                                80, None, 0x7452570003, 0x5EED000003, 0x5AC0000003, n2v_pq=(2.0, 0.5)),
    "metapath-rmat24": Workload("metapath-rmat24", 24, 24, True, False, 5, "metapath", ("its",),
                                100, None, 0x7452570004, 0x5EED000004, 0x5AC0000004, schema_len=5),
    "served-rmat26": Workload("served-rmat26", 26, 16, True, True, 0, "mixed", ("alias", "orej"),
                              80, None, 0x7452570005, 0x5EED000005, 0x5AC0000005, stop_prob=0.2),
}


def make_graph(wl: Workload, scale: Optional[int] = None) -> CSRGraph:
    """The workload's graph; `scale` overrides the vertex count for reduced-size tests."""
    s = wl.scale if scale is None else scale
    g = rmat(s, wl.avg_degree, wl.symmetric, wl.graph_seed)
    if wl.weights or wl.labels:
        attach_attrs(g, wl.graph_seed ^ 0xA77A, weights=wl.weights, labels=wl.labels)
    return g


def make_sources(wl: Workload, g: CSRGraph, nq: Optional[int] = None) -> np.ndarray:
    """One query per vertex (DeepWalk, Node2Vec, MetaPath) or nq uniform sources (PPR)."""
    if nq is None:
        nq = wl.nq
    if nq is None:
        return np.arange(g.n, dtype=np.int32)
    return sources(nq, g.n, wl.src_seed)


def make_schema(wl: Workload) -> np.ndarray:
    """MetaPath schema: schema_len labels drawn with replacement from the label set."""
    return uniform_u32(wl.schema_len, wl.labels, wl.walk_seed ^ 0x5C4E3A).astype(np.uint8)


SERVED_KINDS = ("deepwalk", "ppr", "node2vec")    # request kinds of the served mix, in draw order


def served_requests(wl: Workload, count: int, n: int):
    """The served workload's first `count` requests: sizes uniform in 1..4096, kinds (indexes
    into SERVED_KINDS), query offsets (count + 1) and the sources of all their queries, uniform
    in [0, n).  Every draw depends only on its index, so the first k requests are the same for
    any count."""
    sizes = 1 + uniform_u32(count, 4096, wl.walk_seed ^ 0x5153).astype(np.int64)
    kinds = uniform_u32(count, 3, wl.walk_seed ^ 0xA160).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    return sizes, kinds, offs, sources(int(offs[-1]), n, wl.src_seed)
