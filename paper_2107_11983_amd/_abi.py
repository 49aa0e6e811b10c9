"""ctypes declarations of libtrw.so's C ABI (include/trw.h), same names.

Argument marshalling only: every step of a walk runs in the library's HIP
kernels.  If the library is missing this module raises on import; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrw.so")

TRW_OK, TRW_E_INVALID, TRW_E_UNSUPPORTED, TRW_E_DEVICE = 0, 1, 2, 3
TRW_E_NOMEM_BUDGET, TRW_E_BUSY, TRW_E_TIMEOUT, TRW_E_CANCELLED = 4, 5, 6, 7
STATUS_NAMES = {0: "TRW_OK", 1: "TRW_E_INVALID", 2: "TRW_E_UNSUPPORTED", 3: "TRW_E_DEVICE",
                4: "TRW_E_NOMEM_BUDGET", 5: "TRW_E_BUSY", 6: "TRW_E_TIMEOUT", 7: "TRW_E_CANCELLED"}
TRW_G_SYMMETRIC = 1
TRW_S_NAIVE, TRW_S_ALIAS, TRW_S_ITS, TRW_S_OREJ, TRW_S_REJ = 0, 1, 2, 3, 4
TRW_A_DEEPWALK, TRW_A_PPR, TRW_A_NODE2VEC, TRW_A_METAPATH = 0, 1, 2, 3
TRW_ST_LENGTH, TRW_ST_STOPPED, TRW_ST_DEAD_END, TRW_ST_BAD_SOURCE = 1, 2, 3, 4
TRW_M_PER_STEP, TRW_M_PERSISTENT = 0, 1


class trw_walk_params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_uint32), ("sampler", ctypes.c_uint32),
                ("max_len", ctypes.c_uint32), ("stop_q32", ctypes.c_uint32),
                ("n2v_thr_q16", ctypes.c_uint32 * 3), ("schema_len", ctypes.c_uint32),
                ("schema", ctypes.c_uint8 * 16), ("seed", ctypes.c_uint64)]


class trw_tuning(ctypes.Structure):
    _fields_ = [("walkers_per_lane", ctypes.c_uint32), ("block_threads", ctypes.c_uint32),
                ("blocks_per_cu", ctypes.c_uint32), ("queue_chunk", ctypes.c_uint32),
                ("coop_degree", ctypes.c_uint32), ("no_lds_graph", ctypes.c_uint32),
                ("its_gallop_degree", ctypes.c_uint32), ("n2v_search_degree", ctypes.c_uint32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class trw_server_cfg(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_uint32), ("max_requests", ctypes.c_uint32),
                ("steps_per_tick", ctypes.c_uint32), ("use_hipgraph", ctypes.c_uint32),
                ("serial_ticks", ctypes.c_uint32), ("ring_chunks", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 2)]


TRW_REQ_HOST = 1


class trw_program_params(ctypes.Structure):
    _fields_ = [("max_len", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("user", ctypes.c_uint32 * 16)]


class trw_chunk(ctypes.Structure):
    _fields_ = [("qid_base", ctypes.c_uint64), ("nq", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("lengths", ctypes.c_void_p), ("status", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("entries", ctypes.c_void_p)]


TRW_CHUNK_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(trw_chunk))


class trw_request(ctypes.Structure):
    _fields_ = [("params", trw_walk_params), ("sources", ctypes.c_void_p), ("nq", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("qid_base", ctypes.c_uint64), ("paths", ctypes.c_void_p),
                ("path_stride", ctypes.c_uint64), ("lengths", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("user", ctypes.c_void_p)]


class trw_completion(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_uint64), ("status", ctypes.c_int32), ("nq", ctypes.c_uint32),
                ("user", ctypes.c_void_p), ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64)]


class trw_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("cancelled", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("ticks", ctypes.c_uint64), ("moves", ctypes.c_uint64),
                ("active", ctypes.c_uint32), ("waiting", ctypes.c_uint32), ("pool_bytes", ctypes.c_uint64),
                ("pool_bytes_used", ctypes.c_uint64), ("tick_device_ns", ctypes.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


TRW_DISK_WEIGHTS, TRW_DISK_LABELS = 1, 2


class trw_disk_walk_stats(ctypes.Structure):
    _fields_ = [("runs", ctypes.c_uint64), ("loads", ctypes.c_uint64), ("bytes_read", ctypes.c_uint64),
                ("read_ns", ctypes.c_uint64), ("total_ns", ctypes.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class TrwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(hipcc --offload-arch=gfx950) first")

lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_u32, _u64, _i64, _sz = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_size_t
_st = ctypes.c_int

_SIGS = {
    "trw_last_error": (ctypes.c_char_p, []),
    "trw_abi_version": (_u32, []),
    "trw_graph_create": (_st, [_i64, _i64, _P, _P, _P, _P, _u32, _PP]),
    "trw_graph_validate": (_st, [_P, _P, _sz, _P, ctypes.POINTER(_u64)]),
    "trw_graph_destroy": (_st, [_P]),
    "trw_validate_sources": (_st, [_P, _P, _u64, _P, _sz, _P, ctypes.POINTER(_u64)]),
    "trw_table_bytes": (_st, [_P, _u32, ctypes.POINTER(_sz)]),
    "trw_table_build": (_st, [_P, _u32, _P, _sz, _P, _PP]),
    "trw_table_destroy": (_st, [_P]),
    "trw_walk_workspace_bytes": (_st, [_P, ctypes.POINTER(trw_walk_params), _u64, _u32, ctypes.POINTER(_sz)]),
    "trw_default_tuning": (_st, [_P, ctypes.POINTER(trw_walk_params), _u32, ctypes.POINTER(trw_tuning)]),
    "trw_walk": (_st, [_P, _P, ctypes.POINTER(trw_walk_params), _P, _u64, _u64, _P, _u64, _P, _P, _u32,
                       ctypes.POINTER(trw_tuning), _P, _sz, _P]),
    "trw_walk_noalloc": (_st, [_P, _P, ctypes.POINTER(trw_walk_params), _P, _u64, _u64, _P, _u64, _P, _P, _u32,
                               ctypes.POINTER(trw_tuning), _P]),
    "trw_autotune": (_st, [_P, _P, ctypes.POINTER(trw_walk_params), _P, _u64, _P, _u64, _P, _P, _u32, _u32,
                           _P, _sz, _P, ctypes.POINTER(trw_tuning), ctypes.POINTER(ctypes.c_float)]),
    "trw_adjacency_index_bytes": (_st, [_P, ctypes.POINTER(_sz)]),
    "trw_adjacency_index_build": (_st, [_P, _P, _sz, _P, _PP]),
    "trw_label_index_bytes": (_st, [_P, _u32, ctypes.POINTER(_sz)]),
    "trw_label_index_build": (_st, [_P, _u32, _P, _sz, _P, _PP]),
    "trw_disk_graph_write": (_st, [ctypes.c_char_p, _i64, _i64, _P, _P, _P, _P]),
    "trw_disk_graph_open": (_st, [ctypes.c_char_p, _u64, _PP]),
    "trw_disk_graph_info": (_st, [_P, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(_u32),
                                  ctypes.POINTER(_u32)]),
    "trw_disk_graph_partition": (_st, [_P, _u32, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                       ctypes.POINTER(_i64)]),
    "trw_disk_graph_close": (_st, [_P]),
    "trw_disk_walk_bytes": (_st, [_P, ctypes.POINTER(trw_walk_params), _u64, _u32, ctypes.POINTER(_sz),
                                  ctypes.POINTER(_sz)]),
    "trw_disk_walk": (_st, [_P, ctypes.POINTER(trw_walk_params), _P, _u64, _u64, _P, _u64, _P, _P, _u32, _P, _sz, _P,
                            _sz, ctypes.POINTER(trw_disk_walk_stats), _P]),
    "trw_server_arena_bytes": (_st, [ctypes.POINTER(trw_server_cfg), _sz, ctypes.POINTER(_sz)]),
    "trw_server_create": (_st, [_P, _P, _P, ctypes.POINTER(trw_server_cfg), _P, _sz, _PP]),
    "trw_server_request_bytes": (_st, [_P, ctypes.POINTER(trw_request), ctypes.POINTER(_sz)]),
    "trw_server_submit": (_st, [_P, ctypes.POINTER(trw_request), ctypes.POINTER(_u64)]),
    "trw_server_cancel": (_st, [_P, _u64]),
    "trw_server_poll": (_st, [_P, ctypes.POINTER(trw_completion), _u32, ctypes.POINTER(_u32), _u32]),
    "trw_server_stats_get": (_st, [_P, ctypes.POINTER(trw_server_stats)]),
    "trw_server_destroy": (_st, [_P]),
    "trw_edge_index_bytes": (_st, [_P, ctypes.POINTER(_sz)]),
    "trw_edge_index_build": (_st, [_P, _P, _sz, _P, _PP]),
    "trw_program_check": (_st, [ctypes.c_char_p, ctypes.c_char_p]),
    "trw_program_create": (_st, [ctypes.c_char_p, _PP]),
    "trw_program_kind": (_st, [_P, ctypes.POINTER(_u32)]),
    "trw_program_walk": (_st, [_P, _P, _P, ctypes.POINTER(trw_program_params), _P, _u64, _u64, _P, _u64, _P, _P,
                               _P, _sz, _P]),
    "trw_program_destroy": (_st, [_P]),
    "trw_ppr_end_counts": (_st, [_P, _P, _u64, _P, _P, _u64, _u64, _P, _u64, _P, _P]),
    "trw_topk_workspace_bytes": (_st, [_u64, _u32, ctypes.POINTER(_sz)]),
    "trw_walk_stream_bytes": (_st, [_P, ctypes.POINTER(trw_walk_params), _u32, ctypes.POINTER(_sz),
                                    ctypes.POINTER(_sz)]),
    "trw_walk_stream": (_st, [_P, _P, ctypes.POINTER(trw_walk_params), _P, _u64, _u64, _u32,
                              ctypes.POINTER(trw_tuning), _P, _sz, _P, _sz, TRW_CHUNK_FN, _P, _P]),
    "trw_chunk_to_fd": (ctypes.c_int, [_P, ctypes.POINTER(trw_chunk)]),
    "trw_ppr_walk_counts": (_st, [_P, _P, ctypes.POINTER(trw_walk_params), _P, _u64, _u64, _u64, _P, _u64, _P, _P,
                                  ctypes.POINTER(trw_tuning), _P, _sz, _P]),
    "trw_topk": (_st, [_P, _u64, _u32, _P, _P, _P, _sz, _P]),
    # measurement probe (include/trw_probe.h)
    "trw_probe_fill": (ctypes.c_int, [_P, _u64, _u32, _P]),
    "trw_probe_gather": (ctypes.c_int, [_P, _u64, _u32, _u32, _u32, ctypes.c_int, _u32, _u32, _P, _P]),
    "trw_probe_scatter": (ctypes.c_int, [_P, _u64, _u32, _u32, _u32, _u32, _P]),
    "trw_probe_serve_replay": (ctypes.c_int, [_P, _u32, _P, _P, _P, _u32]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def check(status: int) -> None:
    """Raise TrwError with the library's message unless status == TRW_OK."""
    if status != TRW_OK:
        raise TrwError(status, lib.trw_last_error().decode())


def __getattr__(name):
    if name.startswith("trw_"):
        return getattr(lib, name)
    raise AttributeError(name)


# Module-level functions with the ABI's names (argument marshalling only).
trw_last_error = lib.trw_last_error
trw_abi_version = lib.trw_abi_version
trw_graph_create = lib.trw_graph_create
trw_graph_validate = lib.trw_graph_validate
trw_graph_destroy = lib.trw_graph_destroy
trw_validate_sources = lib.trw_validate_sources
trw_table_bytes = lib.trw_table_bytes
trw_table_build = lib.trw_table_build
trw_table_destroy = lib.trw_table_destroy
trw_walk_workspace_bytes = lib.trw_walk_workspace_bytes
trw_default_tuning = lib.trw_default_tuning
trw_walk = lib.trw_walk
trw_autotune = lib.trw_autotune
trw_adjacency_index_bytes = lib.trw_adjacency_index_bytes
trw_adjacency_index_build = lib.trw_adjacency_index_build
trw_label_index_bytes = lib.trw_label_index_bytes
trw_label_index_build = lib.trw_label_index_build
trw_server_arena_bytes = lib.trw_server_arena_bytes
trw_server_create = lib.trw_server_create
trw_server_request_bytes = lib.trw_server_request_bytes
trw_server_submit = lib.trw_server_submit
trw_server_cancel = lib.trw_server_cancel
trw_server_poll = lib.trw_server_poll
trw_server_stats_get = lib.trw_server_stats_get
trw_server_destroy = lib.trw_server_destroy
trw_program_check = lib.trw_program_check
trw_program_create = lib.trw_program_create
trw_program_kind = lib.trw_program_kind
trw_program_walk = lib.trw_program_walk
trw_program_destroy = lib.trw_program_destroy
trw_ppr_end_counts = lib.trw_ppr_end_counts
trw_topk_workspace_bytes = lib.trw_topk_workspace_bytes
trw_topk = lib.trw_topk
trw_ppr_walk_counts = lib.trw_ppr_walk_counts
trw_walk_stream_bytes = lib.trw_walk_stream_bytes
trw_walk_stream = lib.trw_walk_stream
trw_chunk_to_fd = lib.trw_chunk_to_fd
TRW_CHUNK_TO_FD = TRW_CHUNK_FN(("trw_chunk_to_fd", lib))   # the library's file sink as a chunk function
trw_edge_index_bytes = lib.trw_edge_index_bytes
trw_disk_graph_write = lib.trw_disk_graph_write
trw_disk_graph_open = lib.trw_disk_graph_open
trw_disk_graph_info = lib.trw_disk_graph_info
trw_disk_graph_partition = lib.trw_disk_graph_partition
trw_disk_graph_close = lib.trw_disk_graph_close
trw_disk_walk_bytes = lib.trw_disk_walk_bytes
trw_disk_walk = lib.trw_disk_walk
trw_edge_index_build = lib.trw_edge_index_build
trw_probe_fill = lib.trw_probe_fill
trw_probe_gather = lib.trw_probe_gather
trw_probe_scatter = lib.trw_probe_scatter
trw_probe_serve_replay = lib.trw_probe_serve_replay
