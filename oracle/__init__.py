"""ORACLE — test infrastructure only.

A plain, slow, single-threaded CPU implementation of the ThunderRW walk
method (``trw_oracle.c``, built with gcc into ``liboracle.so``) plus numpy
helpers.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may load it.  It shares no code with the HIP library; the
two meet only through the seeded inputs of ``synth``.

Parameter encoding used here (its own, not the library's):
  algo    : 0 DeepWalk, 1 PPR, 2 Node2Vec, 3 MetaPath
  sampler : 0 NAIVE, 1 ALIAS, 2 ITS, 3 O-REJ, 4 REJ (Node2Vec: O-REJ, REJ on
            weights with the per-vertex bound, or ITS over per-step weights)
  status  : 1 length reached, 2 PPR stop, 3 dead end, 4 source out of range
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

DEEPWALK, PPR, NODE2VEC, METAPATH = 0, 1, 2, 3
NAIVE, ALIAS, ITS, OREJ, REJ = 0, 1, 2, 3, 4
ST_LENGTH, ST_STOPPED, ST_DEAD_END, ST_BAD_SOURCE = 1, 2, 3, 4
ALGOS = {"deepwalk": DEEPWALK, "ppr": PPR, "node2vec": NODE2VEC, "metapath": METAPATH}
SAMPLERS = {"naive": NAIVE, "alias": ALIAS, "its": ITS, "orej": OREJ, "rej": REJ}


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_uint32), ("sampler", ctypes.c_uint32),
                ("max_len", ctypes.c_uint32), ("stop_q32", ctypes.c_uint32),
                ("n2v_thr_q16", ctypes.c_uint32 * 3), ("schema_len", ctypes.c_uint32),
                ("schema", ctypes.c_uint8 * 16), ("seed", ctypes.c_uint64)]


class Counters(ctypes.Structure):
    _fields_ = [("moves", ctypes.c_uint64), ("philox_blocks", ctypes.c_uint64),
                ("its_probes", ctypes.c_uint64), ("orej_trials", ctypes.c_uint64),
                ("adjacency_probes", ctypes.c_uint64), ("label_reads", ctypes.c_uint64),
                ("rej_trials", ctypes.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.trwo_philox4x32_10.restype = None
        lib.trwo_philox4x32_10.argtypes = [P, P, P]
        lib.trwo_alias_build.restype = ctypes.c_int
        lib.trwo_alias_build.argtypes = [ctypes.c_int64, P, P, P, P]
        lib.trwo_its_build.restype = ctypes.c_int
        lib.trwo_its_build.argtypes = [ctypes.c_int64, P, P, P]
        lib.trwo_rej_build.restype = ctypes.c_int
        lib.trwo_rej_build.argtypes = [ctypes.c_int64, P, P, P]
        lib.trwo_walk.restype = ctypes.c_int
        lib.trwo_walk.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, P, ctypes.POINTER(_Params),
                                  P, ctypes.c_int64, ctypes.c_uint64, P, P, ctypes.c_int64, P, P,
                                  ctypes.POINTER(Counters)]
        lib.trwo_end_counts.restype = ctypes.c_int64
        lib.trwo_end_counts.argtypes = [ctypes.c_int64, P, ctypes.c_int64, P, P, ctypes.c_int64,
                                        ctypes.c_int64, P]
        lib.trwo_topk.restype = ctypes.c_int
        lib.trwo_topk.argtypes = [ctypes.c_int64, P, ctypes.c_int64, P, P]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    """One Philox4x32-10 block (Salmon et al., SC 2011): 4 counter words, 2 key words."""
    c = np.ascontiguousarray(np.array(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.array(key, dtype=np.uint32))
    out = np.empty(4, dtype=np.uint32)
    _load().trwo_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def alias_build(row_ptr: np.ndarray, weight: np.ndarray):
    """Integer Vose alias tables: (thr uint32[m], alias int32[m] local indices)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    w = np.ascontiguousarray(weight, dtype=np.uint32)
    m = int(rp[-1])
    thr = np.zeros(m, dtype=np.uint32)
    alias = np.zeros(m, dtype=np.int32)
    rc = _load().trwo_alias_build(len(rp) - 1, _p(rp), _p(w), _p(thr), _p(alias))
    if rc != 0:
        raise RuntimeError(f"trwo_alias_build failed: {rc}")
    return thr, alias


def rej_build(row_ptr: np.ndarray, weight: np.ndarray) -> np.ndarray:
    """REJ's per-vertex bound p*_v: the largest weight of each row (0 if empty)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    w = np.ascontiguousarray(weight, dtype=np.uint32)
    pmax = np.zeros(len(rp) - 1, dtype=np.uint32)
    _load().trwo_rej_build(len(rp) - 1, _p(rp), _p(w), _p(pmax))
    return pmax


def end_counts(n: int, paths: np.ndarray, lengths: np.ndarray, status: np.ndarray, group: int = 0,
               counts: Optional[np.ndarray] = None):
    """PPR end-vertex counts: (counts uint32[groups, n], skipped queries).

    Query i adds one to counts[i // group, paths[i, lengths[i]]] (group 0: one
    row for all queries); queries with a bad source are skipped.
    """
    P = np.ascontiguousarray(paths, dtype=np.int32)
    L = np.ascontiguousarray(lengths, dtype=np.uint32)
    S = np.ascontiguousarray(status, dtype=np.uint8)
    nq = len(L)
    groups = 1 if group <= 0 else max(1, -(-nq // group))
    if counts is None:
        counts = np.zeros((groups, n), dtype=np.uint32)
    assert counts.dtype == np.uint32 and counts.flags.c_contiguous and counts.size >= groups * n
    skipped = _load().trwo_end_counts(n, _p(P), P.shape[1], _p(L), _p(S), nq, group, _p(counts))
    return counts, int(skipped)


def topk(counts: np.ndarray, k: int):
    """The k largest counts (ids int32[k], counts uint32[k]); ties: smaller id first."""
    c = np.ascontiguousarray(counts, dtype=np.uint32).reshape(-1)
    ids = np.zeros(k, dtype=np.int32)
    vals = np.zeros(k, dtype=np.uint32)
    rc = _load().trwo_topk(len(c), _p(c), k, _p(ids), _p(vals))
    if rc != 0:
        raise ValueError(f"trwo_topk failed: {rc}")
    return ids, vals


def its_build(row_ptr: np.ndarray, weight: np.ndarray) -> np.ndarray:
    """Per-row inclusive uint64 prefix sums of the weights."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    w = np.ascontiguousarray(weight, dtype=np.uint32)
    prefix = np.zeros(int(rp[-1]), dtype=np.uint64)
    _load().trwo_its_build(len(rp) - 1, _p(rp), _p(w), _p(prefix))
    return prefix


def n2v_thresholds(p: float, q: float) -> tuple:
    """Q16 acceptance thresholds for Node2Vec darts: p(e)/p* * 2^16, rounded, >= 1.

    p(e) is 1/p when the candidate is the previous vertex, 1 when it is a
    neighbour of it and 1/q otherwise; p* = max(1, 1/p, 1/q).
    """
    weights = (1.0 / p, 1.0, 1.0 / q)
    pstar = max(weights)
    return tuple(max(1, min(65536, int(round(65536.0 * x / pstar)))) for x in weights)


def stop_q32(prob: float) -> int:
    """PPR stop threshold: stop after a move iff r2 < floor(prob * 2^32)."""
    return min(int(prob * 4294967296.0), 0xFFFFFFFF)


@dataclass
class WalkParams:
    algo: int
    sampler: int
    max_len: int
    seed: int
    stop_q32: int = 0
    n2v_thr_q16: tuple = (65536, 65536, 65536)
    schema: tuple = ()

    def to_c(self) -> _Params:
        p = _Params()
        p.algo, p.sampler, p.max_len = self.algo, self.sampler, self.max_len
        p.stop_q32 = self.stop_q32
        for i in range(3):
            p.n2v_thr_q16[i] = self.n2v_thr_q16[i]
        p.schema_len = len(self.schema)
        for i, s in enumerate(self.schema):
            p.schema[i] = int(s)
        p.seed = self.seed & 0xFFFFFFFFFFFFFFFF
        return p


@dataclass
class WalkResult:
    paths: np.ndarray       # int32[nq, max_len+1]; entries past lengths[i] are -1
    lengths: np.ndarray     # uint32[nq]
    status: np.ndarray      # uint8[nq]
    counters: dict = field(default_factory=dict)


def walk(row_ptr, col, params: WalkParams, sources, qid_base: int = 0, qids=None,
         thr=None, alias=None, prefix=None, label=None, weight=None, pmax=None) -> WalkResult:
    """Run every query to completion, one at a time, in query order."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    nq = len(src)
    n = len(rp) - 1
    if params.sampler == ALIAS and (thr is None or alias is None):
        raise ValueError("ALIAS needs thr and alias tables")
    if params.sampler == ITS and params.algo in (DEEPWALK, PPR) and prefix is None:
        raise ValueError("ITS needs the prefix table")
    if params.sampler == REJ:
        if weight is None or pmax is None:
            raise ValueError("REJ needs the weights and the p* table")
        weight = np.ascontiguousarray(weight, dtype=np.uint32)
        pmax = np.ascontiguousarray(pmax, dtype=np.uint32)
    if params.algo == METAPATH and (label is None or not params.schema):
        raise ValueError("MetaPath needs labels and a schema")
    stride = params.max_len + 1
    paths = np.full((nq, stride), -1, dtype=np.int32)
    lengths = np.zeros(nq, dtype=np.uint32)
    status = np.zeros(nq, dtype=np.uint8)
    q = None if qids is None else np.ascontiguousarray(qids, dtype=np.uint64)
    cnt = Counters()
    cp = params.to_c()
    _load().trwo_walk(n, _p(rp), _p(cl), _p(thr), _p(alias), _p(prefix), _p(weight), _p(pmax), _p(label),
                      ctypes.byref(cp), _p(src), nq, qid_base & 0xFFFFFFFFFFFFFFFF, _p(q),
                      _p(paths), stride, _p(lengths), _p(status), ctypes.byref(cnt))
    return WalkResult(paths, lengths, status, cnt.as_dict())
