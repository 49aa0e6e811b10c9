// C ABI of the walk engine: argument checks, handles and dispatch to the
// kernel launchers.  Nothing here computes a walk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "trw_internal.hpp"

struct trw_graph_s {
    trw::GraphDev dev;
    uint32_t flags;
    int device;
};

struct trw_table_s {
    trw_graph graph;
    uint32_t sampler;   // TRW_S_ALIAS / TRW_S_ITS / TRW_S_REJ, or an index kind
    void *buf;
    uint32_t nlab;      // label index: number of labels L
};


static size_t label_index_loff_bytes(const trw::GraphDev &g, uint32_t nlab) {
    const size_t b = sizeof(int32_t) * (size_t)g.n * (nlab + 1);
    return (b + 255) / 256 * 256;
}

// Where a label index's fused entries start (0: the index has none).
static size_t label_index_fused_offset(const trw::GraphDev &g, uint32_t nlab) {
    if (nlab > trw::kMaxFusedLabels) return 0;
    return label_index_loff_bytes(g, nlab) + (sizeof(int32_t) * (size_t)g.m + 255) / 256 * 256;
}

namespace trw {

__global__ void k_zero_first(unsigned long long *p) { *p = 0; }

const GraphDev &graph_dev(trw_graph g) { return g->dev; }

bool table_view(trw_table t, uint32_t kind, const void **buf, trw_graph *graph) {
    if (!t || t->sampler != kind) return false;
    *buf = t->buf;
    *graph = t->graph;
    return true;
}

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

DeviceInfo device_info() {
    static std::mutex mu;
    static std::vector<DeviceInfo> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    for (const auto &d : cache)
        if (d.device == dev) return d;
    DeviceInfo di{dev, 256, 64 * 1024, 64 * 1024};
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
        di.num_cus = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess && v > 0)
        di.lds_per_cu = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
        di.lds_per_block = v;
    cache.push_back(di);
    return di;
}

namespace {

trw_status fail(trw_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

trw_status device_fail(hipError_t e, const char *what) {
    return fail(TRW_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool pair_supported(uint32_t algo, uint32_t sampler) {
    switch (algo) {
        case TRW_A_DEEPWALK:
        case TRW_A_PPR:
            return sampler == TRW_S_NAIVE || sampler == TRW_S_ALIAS || sampler == TRW_S_ITS || sampler == TRW_S_REJ;
        case TRW_A_NODE2VEC:
            return sampler == TRW_S_OREJ;
        case TRW_A_METAPATH:
            return sampler == TRW_S_ITS;
        default:
            return false;
    }
}

trw_status check_params(trw_graph g, const trw_walk_params *p) {
    if (!g) return fail(TRW_E_INVALID, "graph is NULL");
    if (!p) return fail(TRW_E_INVALID, "params is NULL");
    if (p->algo > TRW_A_METAPATH) return fail(TRW_E_UNSUPPORTED, "unknown algorithm");
    if (!pair_supported(p->algo, p->sampler))
        return fail(TRW_E_UNSUPPORTED, "sampler not provided for this algorithm");
    if (p->max_len == 0 || p->max_len > 65535) return fail(TRW_E_INVALID, "max_len must be in 1..65535");
    if (p->algo == TRW_A_NODE2VEC) {
        for (int i = 0; i < 3; ++i)
            if (p->n2v_thr_q16[i] == 0 || p->n2v_thr_q16[i] > 65536)
                return fail(TRW_E_INVALID, "Node2Vec thresholds must be in 1..65536");
    }
    if (p->algo == TRW_A_METAPATH) {
        if (p->schema_len == 0 || p->schema_len > 16) return fail(TRW_E_INVALID, "schema_len must be in 1..16");
        if (!g->dev.label) return fail(TRW_E_INVALID, "MetaPath needs edge labels");
    }
    return TRW_OK;
}

// Defaults measured on MI355X (R-MAT workloads of the benchmark): walks that
// make one random read per move reach the memory system's random-access
// ceiling at low occupancy, where more requests in flight only add
// contention; PPR's short walks also gain from two walkers per lane.
Tuning resolve_tuning(const trw_walk_params *p, uint32_t mode, const trw_tuning *t, bool label_index) {
    const bool static_walk = p->algo == TRW_A_DEEPWALK || p->algo == TRW_A_PPR;
    Tuning tu{1, 256, 8, 256, 256, 1, 0, true};
    if (mode == TRW_M_PERSISTENT) {
        if (static_walk && p->sampler == TRW_S_ALIAS) {
            tu.blocks_per_cu = p->algo == TRW_A_PPR ? 1 : 2;
            tu.walkers_per_lane = p->algo == TRW_A_PPR ? 2 : 1;
        } else if (static_walk && p->sampler == TRW_S_ITS) {
            tu.blocks_per_cu = 4;
        } else if (static_walk && p->sampler == TRW_S_REJ) {
            tu.blocks_per_cu = 2;
        } else if (p->algo == TRW_A_METAPATH && label_index) {
            tu.blocks_per_cu = 2;       // the row scans without an index want the occupancy
            tu.walkers_per_lane = 2;
        }
    }
    if (t) {
        if (t->walkers_per_lane == 1 || t->walkers_per_lane == 2 || t->walkers_per_lane == 4)
            tu.walkers_per_lane = t->walkers_per_lane;
        if (t->block_threads >= 64 && t->block_threads <= 256 && t->block_threads % 64 == 0)
            tu.block_threads = t->block_threads;
        if (t->blocks_per_cu >= 1 && t->blocks_per_cu <= 64) tu.blocks_per_cu = t->blocks_per_cu;
        if (t->queue_chunk >= 1) tu.queue_chunk = t->queue_chunk;
        if (t->coop_degree >= 1) tu.coop_degree = t->coop_degree;
        if (t->its_gallop_degree >= 1) tu.its_gallop_degree = t->its_gallop_degree;
        if (t->n2v_search_degree >= 1) tu.n2v_search_degree = t->n2v_search_degree;
        if (t->no_lds_graph) tu.lds_graph = false;
    }
    return tu;
}

}  // namespace
}  // namespace trw

using namespace trw;

extern "C" {

const char *trw_last_error(void) { return g_last_error.c_str(); }

uint32_t trw_abi_version(void) { return TRW_ABI_VERSION; }

trw_status trw_graph_create(int64_t n, int64_t m, const int32_t *d_row_ptr, const int32_t *d_col,
                            const uint32_t *d_weight, const uint8_t *d_label, uint32_t flags,
                            trw_graph *out) {
    if (!out) return fail(TRW_E_INVALID, "out is NULL");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(TRW_E_INVALID, "n must be in 1..2^31-1");
    if (m < 0 || m >= (int64_t(1) << 31)) return fail(TRW_E_INVALID, "m must be in 0..2^31-1");
    if (!d_row_ptr || (!d_col && m > 0)) return fail(TRW_E_INVALID, "row_ptr / col is NULL");
    auto *g = new (std::nothrow) trw_graph_s;
    if (!g) return fail(TRW_E_INVALID, "out of host memory");
    g->dev = GraphDev{d_row_ptr, d_col, d_weight, d_label, (int32_t)n, (int32_t)m,
                      (flags & TRW_G_SYMMETRIC) ? 1 : 0};
    g->flags = flags;
    g->device = device_info().device;
    *out = g;
    return TRW_OK;
}

trw_status trw_graph_validate(trw_graph g, void *d_ws, size_t ws_bytes, trw_stream_t stream, uint64_t *n_bad) {
    if (!g || !n_bad) return fail(TRW_E_INVALID, "graph / n_bad is NULL");
    if (!d_ws || ws_bytes < 64 || (reinterpret_cast<uintptr_t>(d_ws) & 7))
        return fail(TRW_E_INVALID, "validate needs >= 64 bytes of 8-byte aligned device scratch");
    auto s = static_cast<hipStream_t>(stream);
    auto *bad = static_cast<unsigned long long *>(d_ws);
    hipError_t e = launch_validate(g->dev, bad, s);
    if (e != hipSuccess) return device_fail(e, "validate launch");
    unsigned long long h = 0;
    e = hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(e, "validate readback");
    *n_bad = h;
    if (h) return fail(TRW_E_INVALID, "graph failed validation: " + std::to_string(h) + " violations");
    if (g->dev.symmetric) {   // only on a well-formed graph: the check reads the rows it is pointed to
        unsigned long long *bad2 = bad + 1;
        hipLaunchKernelGGL(k_zero_first, dim3(1), dim3(1), 0, s, bad2);
        e = launch_symmetry_check(g->dev, bad2, s);
        if (e != hipSuccess) return device_fail(e, "symmetry check launch");
        e = hipMemcpyAsync(&h, bad2, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return device_fail(e, "symmetry check readback");
        *n_bad = h;
        if (h) return fail(TRW_E_INVALID, "graph flagged symmetric has " + std::to_string(h) + " edges without reverse");
    }
    return TRW_OK;
}

trw_status trw_graph_destroy(trw_graph g) {
    delete g;
    return TRW_OK;
}

trw_status trw_validate_sources(trw_graph g, const int32_t *d_sources, uint64_t nq, void *d_ws, size_t ws_bytes,
                                trw_stream_t stream, uint64_t *n_bad) {
    if (!g || !n_bad) return fail(TRW_E_INVALID, "graph / n_bad is NULL");
    if (nq >= (uint64_t(1) << 32)) return fail(TRW_E_INVALID, "nq must be < 2^32");
    if (nq > 0 && !d_sources) return fail(TRW_E_INVALID, "sources is NULL");
    if (!d_ws || ws_bytes < 8 || (reinterpret_cast<uintptr_t>(d_ws) & 7))
        return fail(TRW_E_INVALID, "validate_sources needs >= 8 bytes of 8-byte aligned device scratch");
    auto s = static_cast<hipStream_t>(stream);
    auto *bad = static_cast<unsigned long long *>(d_ws);
    hipError_t e = launch_validate_sources(d_sources, nq, g->dev.n, bad, s);
    if (e != hipSuccess) return device_fail(e, "validate_sources launch");
    unsigned long long h = 0;
    e = hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(e, "validate_sources readback");
    *n_bad = h;
    if (h) return fail(TRW_E_INVALID, std::to_string(h) + " sources outside [0, n)");
    return TRW_OK;
}

trw_status trw_table_bytes(trw_graph g, uint32_t sampler, size_t *bytes) {
    if (!g || !bytes) return fail(TRW_E_INVALID, "graph / bytes is NULL");
    switch (sampler) {
        case TRW_S_ALIAS: *bytes = kAliasEntryBytes * (size_t)g->dev.m; return TRW_OK;
        case TRW_S_ITS:
            *bytes = its_prefix_bytes(g->dev.m) + its_next_bytes(g->dev.m) + sizeof(uint64_t) * (size_t)g->dev.n;
            return TRW_OK;
        case TRW_S_REJ: *bytes = rej_records_bytes(g->dev.m) + sizeof(uint32_t) * (size_t)g->dev.n; return TRW_OK;
        case TRW_S_NAIVE:
        case TRW_S_OREJ: *bytes = 0; return fail(TRW_E_UNSUPPORTED, "sampler has no table");
        default: return fail(TRW_E_UNSUPPORTED, "unknown sampler");
    }
}

trw_status trw_table_build(trw_graph g, uint32_t sampler, void *d_buf, size_t bytes, trw_stream_t stream,
                           trw_table *out) {
    if (!g || !out) return fail(TRW_E_INVALID, "graph / out is NULL");
    size_t need = 0;
    trw_status st = trw_table_bytes(g, sampler, &need);
    if (st != TRW_OK) return st;
    if (!g->dev.weight) return fail(TRW_E_INVALID, "table needs edge weights");
    if (bytes < need) return fail(TRW_E_INVALID, "table buffer too small");
    if ((g->dev.m > 0 || sampler != TRW_S_ALIAS) && (!d_buf || (reinterpret_cast<uintptr_t>(d_buf) & 31)))
        return fail(TRW_E_INVALID, "table buffer NULL or not 32-byte aligned");
    // the ITS search reads whole 64-byte blocks of the prefix array, whose parts
    // are laid out at 256-byte offsets from the base
    if (sampler == TRW_S_ITS && (reinterpret_cast<uintptr_t>(d_buf) & 255))
        return fail(TRW_E_INVALID, "ITS table buffer not 256-byte aligned");
    auto s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    char *base = static_cast<char *>(d_buf);
    if (sampler == TRW_S_REJ) {
        e = launch_rej_build(g->dev, static_cast<uint4 *>(d_buf),
                             reinterpret_cast<uint32_t *>(base + rej_records_bytes(g->dev.m)), s);
    } else if (sampler == TRW_S_ITS) {
        const size_t pb = its_prefix_bytes(g->dev.m);
        e = launch_its_build(g->dev, static_cast<uint64_t *>(d_buf), reinterpret_cast<uint4 *>(base + pb),
                             reinterpret_cast<uint64_t *>(base + pb + its_next_bytes(g->dev.m)), s);
    } else if (g->dev.m > 0) {
        e = launch_alias_build(g->dev, static_cast<uint4 *>(d_buf), s);
    }
    if (e != hipSuccess) return device_fail(e, "table build launch");
    auto *t = new (std::nothrow) trw_table_s{g, sampler, d_buf, 0};
    if (!t) return fail(TRW_E_INVALID, "out of host memory");
    *out = t;
    return TRW_OK;
}

trw_status trw_label_index_bytes(trw_graph g, uint32_t n_labels, size_t *bytes) {
    if (!g || !bytes) return fail(TRW_E_INVALID, "graph / bytes is NULL");
    if (n_labels == 0 || n_labels > kMaxIndexLabels) return fail(TRW_E_INVALID, "n_labels must be in 1..64");
    const size_t fused = label_index_fused_offset(g->dev, n_labels);
    *bytes = fused ? fused + 2 * sizeof(uint4) * (size_t)g->dev.m
                   : label_index_loff_bytes(g->dev, n_labels) + sizeof(int32_t) * (size_t)g->dev.m;
    return TRW_OK;
}

trw_status trw_label_index_build(trw_graph g, uint32_t n_labels, void *d_buf, size_t bytes, trw_stream_t stream,
                                 trw_table *out) {
    if (!g || !out) return fail(TRW_E_INVALID, "graph / out is NULL");
    size_t need = 0;
    trw_status st = trw_label_index_bytes(g, n_labels, &need);
    if (st != TRW_OK) return st;
    if (!g->dev.label) return fail(TRW_E_INVALID, "label index needs edge labels");
    if (bytes < need) return fail(TRW_E_INVALID, "label index buffer too small");
    if (!d_buf || (reinterpret_cast<uintptr_t>(d_buf) & 255))
        return fail(TRW_E_INVALID, "label index buffer NULL or not 256-byte aligned");
    auto *loff = static_cast<int32_t *>(d_buf);
    auto *lcol = reinterpret_cast<int32_t *>(static_cast<char *>(d_buf) + label_index_loff_bytes(g->dev, n_labels));
    hipError_t e = launch_label_index_build(g->dev, n_labels, loff, lcol, static_cast<hipStream_t>(stream));
    const size_t fused = label_index_fused_offset(g->dev, n_labels);
    if (e == hipSuccess && fused)
        e = launch_label_fused_build(g->dev, n_labels, loff, lcol,
                                     reinterpret_cast<uint4 *>(static_cast<char *>(d_buf) + fused),
                                     static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_fail(e, "label index build launch");
    auto *t = new (std::nothrow) trw_table_s{g, kLabelIndexKind, d_buf, n_labels};
    if (!t) return fail(TRW_E_INVALID, "out of host memory");
    *out = t;
    return TRW_OK;
}

trw_status trw_adjacency_index_bytes(trw_graph g, size_t *bytes) {
    if (!g || !bytes) return fail(TRW_E_INVALID, "graph / bytes is NULL");
    *bytes = sizeof(uint4) * (size_t)g->dev.m;
    return TRW_OK;
}

trw_status trw_adjacency_index_build(trw_graph g, void *d_buf, size_t bytes, trw_stream_t stream, trw_table *out) {
    if (!g || !out) return fail(TRW_E_INVALID, "graph / out is NULL");
    if (bytes < sizeof(uint4) * (size_t)g->dev.m) return fail(TRW_E_INVALID, "adjacency index buffer too small");
    if (g->dev.m > 0 && (!d_buf || (reinterpret_cast<uintptr_t>(d_buf) & 15)))
        return fail(TRW_E_INVALID, "adjacency index buffer NULL or not 16-byte aligned");
    if (g->dev.m > 0) {
        hipError_t e = launch_adjacency_build(g->dev, static_cast<uint4 *>(d_buf), static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return device_fail(e, "adjacency index build launch");
    }
    auto *t = new (std::nothrow) trw_table_s{g, kAdjacencyKind, d_buf, 0};
    if (!t) return fail(TRW_E_INVALID, "out of host memory");
    *out = t;
    return TRW_OK;
}

trw_status trw_edge_index_bytes(trw_graph g, size_t *bytes) {
    if (!g || !bytes) return fail(TRW_E_INVALID, "graph / bytes is NULL");
    *bytes = edge_index_records_bytes(g->dev.m) + sizeof(unsigned long long) * eset_slots(g->dev.m);
    return TRW_OK;
}

trw_status trw_edge_index_build(trw_graph g, void *d_buf, size_t bytes, trw_stream_t stream, trw_table *out) {
    if (!g || !out) return fail(TRW_E_INVALID, "graph / out is NULL");
    const size_t rec = edge_index_records_bytes(g->dev.m);
    const unsigned long long slots = eset_slots(g->dev.m);
    if (bytes < rec + sizeof(unsigned long long) * slots) return fail(TRW_E_INVALID, "edge index buffer too small");
    if (!d_buf || (reinterpret_cast<uintptr_t>(d_buf) & 255))
        return fail(TRW_E_INVALID, "edge index buffer NULL or not 256-byte aligned");
    // The hash set is filled with device atomics, which host memory across
    // the host link does not promise to support.
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, d_buf) == hipSuccess) {
        if (attr.type == hipMemoryTypeHost)
            return fail(TRW_E_UNSUPPORTED, "the edge index must be built in device memory");
    } else {
        (void)hipGetLastError();   // a pointer the runtime does not know: left to the launch
    }
    auto s = static_cast<hipStream_t>(stream);
    hipError_t e = g->dev.m > 0 ? launch_adjacency_build(g->dev, static_cast<uint4 *>(d_buf), s) : hipSuccess;
    if (e == hipSuccess)
        e = launch_edge_set_build(g->dev, reinterpret_cast<unsigned long long *>(static_cast<char *>(d_buf) + rec),
                                  slots, s);
    if (e != hipSuccess) return device_fail(e, "edge index build launch");
    auto *t = new (std::nothrow) trw_table_s{g, kEdgeIndexKind, d_buf, 0};
    if (!t) return fail(TRW_E_INVALID, "out of host memory");
    *out = t;
    return TRW_OK;
}

trw_status trw_table_destroy(trw_table t) {
    delete t;
    return TRW_OK;
}

trw_status trw_walk_workspace_bytes(trw_graph g, const trw_walk_params *p, uint64_t nq, uint32_t mode,
                                    size_t *bytes) {
    trw_status st = check_params(g, p);
    if (st != TRW_OK) return st;
    if (!bytes) return fail(TRW_E_INVALID, "bytes is NULL");
    if (mode > TRW_M_PERSISTENT) return fail(TRW_E_INVALID, "unknown mode");
    if (nq >= (uint64_t(1) << 32)) return fail(TRW_E_INVALID, "nq must be < 2^32");
    *bytes = walk_workspace_bytes(mode, nq, p->max_len);
    return TRW_OK;
}

trw_status trw_default_tuning(trw_graph g, const trw_walk_params *p, uint32_t mode, trw_tuning *out) {
    trw_status st = check_params(g, p);
    if (st != TRW_OK) return st;
    if (!out) return fail(TRW_E_INVALID, "out is NULL");
    const Tuning tu = resolve_tuning(p, mode, nullptr, false);
    std::memset(out, 0, sizeof(*out));
    out->walkers_per_lane = tu.walkers_per_lane;
    out->block_threads = tu.block_threads;
    out->blocks_per_cu = tu.blocks_per_cu;
    out->queue_chunk = tu.queue_chunk;
    out->coop_degree = tu.coop_degree;
    out->its_gallop_degree = tu.its_gallop_degree;
    out->n2v_search_degree = tu.n2v_search_degree;
    return TRW_OK;
}

}  // extern "C"

namespace {

// trw_walk, and with d_counts the PPR estimate walk (no paths: each query's
// end vertex is counted instead).
trw_status walk_impl(trw_graph g, trw_table table, const trw_walk_params *p, const int32_t *d_sources,
                     uint64_t nq, uint64_t qid_base, int32_t *d_paths, uint64_t path_stride,
                     uint32_t *d_lengths, uint8_t *d_status, uint32_t mode, const trw_tuning *tuning,
                     void *d_ws, size_t ws_bytes, trw_stream_t stream, uint32_t *d_counts, uint64_t group,
                     uint64_t counts_len) {
    trw_status st = check_params(g, p);
    if (st != TRW_OK) return st;
    const bool counts = d_counts != nullptr;
    if (counts) {
        if (p->algo != TRW_A_PPR) return fail(TRW_E_UNSUPPORTED, "end-vertex counting walks are PPR walks");
        const uint64_t groups = group ? (nq + group - 1) / group : 1;
        if (counts_len < std::max<uint64_t>(groups, 1) * (uint64_t)g->dev.n)
            return fail(TRW_E_INVALID, "counts holds fewer than groups * n entries");
    }
    if (mode > TRW_M_PERSISTENT) return fail(TRW_E_INVALID, "unknown mode");
    if (nq >= (uint64_t(1) << 32)) return fail(TRW_E_INVALID, "nq must be < 2^32");
    const bool needs_table = (p->algo == TRW_A_DEEPWALK || p->algo == TRW_A_PPR) &&
                             (p->sampler == TRW_S_ALIAS || p->sampler == TRW_S_ITS || p->sampler == TRW_S_REJ);
    if (needs_table) {
        if (!table) return fail(TRW_E_INVALID, "ALIAS / ITS / REJ walks need a table");
        if (table->graph != g) return fail(TRW_E_INVALID, "table was built for another graph");
        if (table->sampler != p->sampler) return fail(TRW_E_INVALID, "table was built for another sampler");
    }
    const bool adjacency = !needs_table && p->algo != TRW_A_METAPATH && table != nullptr;
    if (adjacency) {
        if (table->graph != g) return fail(TRW_E_INVALID, "adjacency index was built for another graph");
        if (table->sampler != kAdjacencyKind && table->sampler != kEdgeIndexKind)
            return fail(TRW_E_INVALID, "NAIVE / OREJ walks take an adjacency or edge index, or no table");
    }
    const bool label_index = p->algo == TRW_A_METAPATH && table != nullptr;
    if (label_index) {
        if (table->graph != g) return fail(TRW_E_INVALID, "label index was built for another graph");
        if (table->sampler != kLabelIndexKind) return fail(TRW_E_INVALID, "MetaPath takes a label index or no table");
        for (uint32_t i = 0; i < p->schema_len; ++i)
            if (p->schema[i] >= table->nlab) return fail(TRW_E_INVALID, "schema label >= label index n_labels");
    }
    if (!counts && path_stride < (uint64_t)p->max_len + 1) return fail(TRW_E_INVALID, "path_stride < max_len + 1");
    if (nq == 0) return TRW_OK;
    if (!d_sources || (!counts && !d_paths) || (!counts && (!d_lengths || !d_status)) ||
        (counts && (d_lengths == nullptr) != (d_status == nullptr)))
        return fail(TRW_E_INVALID, "sources / paths / lengths / status is NULL");
    const size_t need = walk_workspace_bytes(mode, nq, p->max_len);
    if (!d_ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_ws) & 255))
        return fail(TRW_E_INVALID, "workspace NULL, too small or not 256-byte aligned");

    WalkDev w{};
    w.max_len = p->max_len;
    w.stop_q32 = p->algo == TRW_A_PPR ? p->stop_q32 : 0;
    for (int i = 0; i < 3; ++i) w.thr[i] = p->n2v_thr_q16[i];
    w.schema_len = p->algo == TRW_A_METAPATH ? p->schema_len : 1;
    for (int i = 0; i < 8; ++i) {
        w.schema_lo |= (uint64_t)p->schema[i] << (8 * i);
        w.schema_hi |= (uint64_t)p->schema[8 + i] << (8 * i);
    }
    w.seed = p->seed;
    w.sources = d_sources;
    w.nq = (uint32_t)nq;
    w.qid_base = qid_base;
    w.paths = d_paths;
    w.stride = path_stride;
    w.lengths = d_lengths;
    w.status = d_status;
    w.end_counts = d_counts;
    w.end_group = group;
    TableDev t{nullptr, nullptr, nullptr, nullptr, 0, nullptr};
    if (adjacency) t.adj = static_cast<const uint4 *>(table->buf);
    if (adjacency && table->sampler == kEdgeIndexKind) {
        t.eset = reinterpret_cast<const unsigned long long *>(static_cast<const char *>(table->buf) +
                                                              edge_index_records_bytes(g->dev.m));
        t.eset_mask = eset_slots(g->dev.m) - 1;
    }
    if (needs_table) {
        if (p->sampler == TRW_S_ALIAS) {
            t.alias = static_cast<const uint4 *>(table->buf);
        } else if (p->sampler == TRW_S_REJ) {
            t.rej = static_cast<const uint4 *>(table->buf);
            t.pmax = reinterpret_cast<const uint32_t *>(static_cast<const char *>(table->buf) +
                                                        rej_records_bytes(g->dev.m));
        } else {
            const char *base = static_cast<const char *>(table->buf);
            t.prefix = static_cast<const uint64_t *>(table->buf);
            t.its_next = reinterpret_cast<const uint4 *>(base + its_prefix_bytes(g->dev.m));
            t.its_w = reinterpret_cast<const uint64_t *>(base + its_prefix_bytes(g->dev.m) + its_next_bytes(g->dev.m));
        }
    }
    if (label_index) {
        t.loff = static_cast<const int32_t *>(table->buf);
        t.lcol = reinterpret_cast<const int32_t *>(static_cast<const char *>(table->buf) +
                                                   label_index_loff_bytes(g->dev, table->nlab));
        t.nlab = table->nlab;
        if (const size_t fused = label_index_fused_offset(g->dev, table->nlab))
            t.lfused = reinterpret_cast<const uint4 *>(static_cast<const char *>(table->buf) + fused);
    }
    const Tuning tu = resolve_tuning(p, mode, tuning, label_index);
    w.its_gallop = tu.its_gallop_degree;
    w.n2v_search = tu.n2v_search_degree;
    hipError_t e = counts ? launch_ppr_counts(g->dev, t, p->sampler, w, tu, device_info(), d_ws,
                                              static_cast<hipStream_t>(stream))
                          : launch_walk(g->dev, t, p->algo, p->sampler, w, mode, tu, device_info(), d_ws, ws_bytes,
                                        static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_fail(e, "walk launch");
    return TRW_OK;
}

}  // namespace

extern "C" {

trw_status trw_walk(trw_graph g, trw_table table, const trw_walk_params *p, const int32_t *d_sources,
                    uint64_t nq, uint64_t qid_base, int32_t *d_paths, uint64_t path_stride,
                    uint32_t *d_lengths, uint8_t *d_status, uint32_t mode, const trw_tuning *tuning,
                    void *d_ws, size_t ws_bytes, trw_stream_t stream) {
    return walk_impl(g, table, p, d_sources, nq, qid_base, d_paths, path_stride, d_lengths, d_status, mode, tuning,
                     d_ws, ws_bytes, stream, nullptr, 0, 0);
}


}  // extern "C"

namespace {

// Workspace of trw_walk_noalloc: a device array in this library's code object,
// one copy per GPU.  In host code its name is only a stand-in for the symbol;
// the device address comes from hipGetSymbolAddress, looked up once per device
// (with that device current) and kept.
__device__ __align__(256) unsigned char scratch[TRW_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxScratchDevices] = {};

trw_status scratch_of_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(TRW_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return device_fail(e, "hipGetSymbolAddress(scratch)");
        scratch_ptr[dev] = ptr;
    }
    *out = scratch_ptr[dev];
    return TRW_OK;
}

}  // namespace

extern "C" {

trw_status trw_walk_noalloc(trw_graph g, trw_table table, const trw_walk_params *p, const int32_t *d_sources,
                            uint64_t nq, uint64_t qid_base, int32_t *d_paths, uint64_t path_stride,
                            uint32_t *d_lengths, uint8_t *d_status, uint32_t mode, const trw_tuning *tuning,
                            trw_stream_t stream) {
    if (!g || !p) return fail(TRW_E_INVALID, "graph / params is NULL");
    if (mode > TRW_M_PERSISTENT) return fail(TRW_E_INVALID, "unknown mode");
    const size_t need = walk_workspace_bytes(mode, nq, p->max_len);
    if (need > TRW_NOALLOC_SCRATCH_BYTES)
        return fail(TRW_E_INVALID, "the walk needs " + std::to_string(need) +
                                       " bytes of workspace; trw_walk_noalloc holds " +
                                       std::to_string((size_t)TRW_NOALLOC_SCRATCH_BYTES) +
                                       " (use trw_walk with a caller workspace)");
    void *ws = nullptr;
    trw_status st = scratch_of_current_device(&ws);
    if (st != TRW_OK) return st;
    return walk_impl(g, table, p, d_sources, nq, qid_base, d_paths, path_stride, d_lengths, d_status, mode, tuning,
                     ws, TRW_NOALLOC_SCRATCH_BYTES, stream, nullptr, 0, 0);
}

trw_status trw_ppr_walk_counts(trw_graph g, trw_table table, const trw_walk_params *p, const int32_t *d_sources,
                               uint64_t nq, uint64_t qid_base, uint64_t group, uint32_t *d_counts,
                               uint64_t counts_len, uint32_t *d_lengths, uint8_t *d_status,
                               const trw_tuning *tuning, void *d_ws, size_t ws_bytes, trw_stream_t stream) {
    if (!d_counts) return fail(TRW_E_INVALID, "counts is NULL");
    return walk_impl(g, table, p, d_sources, nq, qid_base, nullptr, 0, d_lengths, d_status, TRW_M_PERSISTENT,
                     tuning, d_ws, ws_bytes, stream, d_counts, group, counts_len);
}

trw_status trw_autotune(trw_graph g, trw_table table, const trw_walk_params *p, const int32_t *d_sources,
                        uint64_t nq, int32_t *d_paths, uint64_t path_stride, uint32_t *d_lengths,
                        uint8_t *d_status, uint32_t mode, uint32_t budget, void *d_ws, size_t ws_bytes,
                        trw_stream_t stream, trw_tuning *out, float *best_ms) {
    if (!out) return fail(TRW_E_INVALID, "out is NULL");
    // Candidates: the launch shape (walkers per lane, blocks per CU), the queue
    // chunk, and for MetaPath without a label index the degree at which a row
    // is scanned by the whole wave.  The library default comes first, so a
    // budget of 1 returns it.  A second phase then tries the degree thresholds
    // of the walk, if it has one, with the best launch shape of the first: the
    // row degree from which ITS searches from its guess (shorter rows bisect),
    // and the degree up to which Node2Vec's adjacency test searches the
    // previous vertex's row instead of probing the edge index.
    std::vector<trw_tuning> cands;
    const bool scans = p->algo == TRW_A_METAPATH && table == nullptr;
    const bool its_walk = (p->algo == TRW_A_DEEPWALK || p->algo == TRW_A_PPR) && p->sampler == TRW_S_ITS;
    const bool n2v_eset = p->algo == TRW_A_NODE2VEC && table != nullptr && table->sampler == kEdgeIndexKind;
    if (mode == TRW_M_PERSISTENT) {
        const Tuning d = resolve_tuning(p, mode, nullptr, p->algo == TRW_A_METAPATH && table != nullptr);
        trw_tuning def{};
        def.walkers_per_lane = d.walkers_per_lane; def.block_threads = d.block_threads;
        def.blocks_per_cu = d.blocks_per_cu; def.queue_chunk = d.queue_chunk; def.coop_degree = d.coop_degree;
        def.its_gallop_degree = d.its_gallop_degree; def.n2v_search_degree = d.n2v_search_degree;
        cands.push_back(def);
        for (uint32_t wpl : {1u, 2u, 4u})
            for (uint32_t bpc : {1u, 2u, 4u, 8u})
                for (uint32_t chunk : {128u, 256u})
                    for (uint32_t coop : {256u, 1024u, 4096u, 16384u}) {
                        if (!scans && coop != 256u) continue;
                        trw_tuning t = def;
                        t.walkers_per_lane = wpl; t.block_threads = 256; t.blocks_per_cu = bpc;
                        t.queue_chunk = chunk; t.coop_degree = coop;
                        cands.push_back(t);
                    }
    } else {
        const Tuning d = resolve_tuning(p, mode, nullptr, false);
        for (uint32_t bpc : {2u, 4u, 8u, 16u})
            for (uint32_t threads : {128u, 256u}) {
                trw_tuning t{};
                t.walkers_per_lane = 1; t.block_threads = threads; t.blocks_per_cu = bpc;
                t.queue_chunk = 256; t.coop_degree = 256;
                t.its_gallop_degree = d.its_gallop_degree; t.n2v_search_degree = d.n2v_search_degree;
                cands.push_back(t);
            }
    }
    std::vector<uint32_t> degrees;       // second phase: values of the walk's threshold
    if (its_walk) degrees = {8u, 64u, 512u};
    else if (n2v_eset) degrees = {4u, 16u, 64u};
    const size_t limit = budget > 0 ? budget : cands.size() + degrees.size();
    if (cands.size() > limit) cands.resize(limit);
    auto s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(TRW_E_DEVICE, "hipEventCreate failed");
    // The default (first candidate) is kept unless another beats it by 3%: a
    // sample's timings differ by a few percent from run to run, and a choice
    // within that noise does not carry over to the whole batch.
    constexpr float kMargin = 0.97f;
    float best = -1.0f, default_ms = -1.0f;
    trw_tuning best_t{};
    trw_status result = TRW_OK;
    auto try_candidate = [&](const trw_tuning &c) {
        // one untimed run (warm caches), one timed run
        for (int rep = 0; rep < 2 && result == TRW_OK; ++rep) {
            (void)hipEventRecord(e0, s);
            result = trw_walk(g, table, p, d_sources, nq, 0, d_paths, path_stride, d_lengths, d_status, mode,
                              &c, d_ws, ws_bytes, stream);
            (void)hipEventRecord(e1, s);
        }
        if (result != TRW_OK) return;
        if (hipEventSynchronize(e1) != hipSuccess) { result = fail(TRW_E_DEVICE, "event sync failed"); return; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (best < 0) {
            best = default_ms = ms;
            best_t = c;
        } else if (ms < best && ms < kMargin * default_ms) {
            best = ms;
            best_t = c;
        }
    };
    for (const auto &c : cands) {
        try_candidate(c);
        if (result != TRW_OK) break;
    }
    const trw_tuning shape = best_t;
    for (size_t i = 0; i < degrees.size() && cands.size() + i < limit && result == TRW_OK; ++i) {
        trw_tuning c = shape;
        if (its_walk) c.its_gallop_degree = degrees[i];
        else c.n2v_search_degree = degrees[i];
        try_candidate(c);
    }
    // Confirm a winner against the default: five alternating timings of the
    // two (after a warm run of each); the winner is kept only if its median is
    // again at least 3% below the default's, so a sample that favoured it by
    // chance does not carry the choice.
    const bool is_default = std::memcmp(&best_t, &cands[0], sizeof(trw_tuning)) == 0;
    if (result == TRW_OK && !is_default) {
        std::vector<float> t_def, t_best;
        for (int rep = 0; rep < 6 && result == TRW_OK; ++rep) {
            for (int which = 0; which < 2 && result == TRW_OK; ++which) {
                const trw_tuning &c = which == 0 ? cands[0] : best_t;
                (void)hipEventRecord(e0, s);
                result = trw_walk(g, table, p, d_sources, nq, 0, d_paths, path_stride, d_lengths, d_status, mode,
                                  &c, d_ws, ws_bytes, stream);
                (void)hipEventRecord(e1, s);
                if (result != TRW_OK) break;
                if (hipEventSynchronize(e1) != hipSuccess) { result = fail(TRW_E_DEVICE, "event sync failed"); break; }
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) (which == 0 ? t_def : t_best).push_back(ms);
            }
        }
        if (result == TRW_OK) {
            std::sort(t_def.begin(), t_def.end());
            std::sort(t_best.begin(), t_best.end());
            const float med_def = t_def[t_def.size() / 2], med_best = t_best[t_best.size() / 2];
            if (med_best < kMargin * med_def) {
                best = med_best;
            } else {
                best_t = cands[0];
                best = med_def;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != TRW_OK) return result;
    *out = best_t;
    if (best_ms) *best_ms = best;
    return TRW_OK;
}

}  // extern "C"
