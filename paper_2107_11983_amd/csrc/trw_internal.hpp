// Internal types shared by the C ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/trw.h"
#include "trw_device.hpp"

namespace trw {

// Device view of a CSR graph (borrowed caller memory).
struct GraphDev {
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *weight;
    const uint8_t *label;
    int32_t n;
    int32_t m;
    int32_t symmetric;   // every edge has its reverse (checked by trw_graph_validate)
};

// An ALIAS entry is 32 bytes, two uint4 per edge slot:
//   [0] {thr, dst_first, dst_second, 0}
//   [1] {row_off(dst_first), deg(dst_first), row_off(dst_second), deg(dst_second)}
// The destination ids and their row ranges sit beside the coin threshold, so
// a move reads one 32-byte entry (one cache line) and neither the adjacency
// array nor the row offsets.
// MetaPath label index: each row stably sorted by label (so within one label
// the CSR order is kept) in lcol, and per vertex v the offsets
// loff[v * (L + 1) + x] = start in lcol of v's edges with label x, for
// x = 0..L (loff[v][L] = end of the row).  Edges with labels >= L are left
// out: a schema label is always < L, so they never match.
struct TableDev {
    const uint4 *alias;       // ALIAS: 2 x uint4 per edge slot
    const uint64_t *prefix;   // ITS: inclusive prefix per row
    const uint4 *its_next;    // ITS: 2 x uint4 per edge slot {dst, row_off(dst), deg(dst), 0}, {W(dst) lo, hi, 0, 0}
    const uint64_t *its_w;    // ITS: W per vertex (its row's weight sum)
    const int32_t *loff;      // label index: (L + 1) offsets per vertex
    const int32_t *lcol;      // label index: label-sorted destinations
    uint32_t nlab;            // label index: L
    const uint4 *adj;         // adjacency index: {dst, row_off(dst), deg(dst), 0} per edge slot
    const unsigned long long *eset;   // edge index: hash set of the edges (u, v) as u << 32 | v
    unsigned long long eset_mask;     // its slot count - 1 (a power of two)
    const uint4 *rej;         // REJ: 2 x uint4 per edge slot {w, dst, row_off(dst), deg(dst)}, {p*(dst), 0, 0, 0}
    const uint32_t *pmax;     // REJ: p*_v per vertex
    const uint4 *lfused;      // label index with L <= kMaxFusedLabels: 2 x uint4 per destination slot
                              // {lcol[e], loff[lcol[e]][0..L]} (unused offsets 0)
};

// Edge hash set slots: at most half full (kEsetEmpty and eset_hash are in
// trw_device.hpp, shared with walk programs).
__host__ __device__ inline unsigned long long eset_slots(int64_t m) {
    unsigned long long cap = 64;
    while (cap < 2ull * (unsigned long long)m) cap <<= 1;
    return cap;
}
constexpr size_t kAliasEntryBytes = 32;
constexpr uint32_t kMaxIndexLabels = 64;
// Label indexes over at most this many labels also hold fused entries: a
// destination and its L + 1 label offsets in 32 bytes.
constexpr uint32_t kMaxFusedLabels = 6;

// Parameters of one batch of queries as the kernels see them.
struct WalkDev {
    uint32_t max_len;
    uint32_t stop_q32;
    uint32_t thr[3];
    uint32_t schema_len;
    uint64_t schema_lo;      // labels 0..7 of the MetaPath schema, one byte each
    uint64_t schema_hi;      // labels 8..15
    uint64_t seed;
    const int32_t *sources;
    uint32_t nq;
    uint64_t qid_base;
    int32_t *paths;
    uint64_t stride;
    uint32_t *lengths;
    uint8_t *status;
    uint32_t *end_counts;     // PPR estimate walks: counts[(qi / end_group) * n + end vertex]
    uint64_t end_group;       // queries per counts row (0: one row)
    uint32_t its_gallop;      // ITS: rows of at least this many slots search from the guess (0, 1: all)
    uint32_t n2v_search;      // Node2Vec with an edge index: prev rows of at most this many
                              // edges are searched instead of probing the hash set (0: none)
};

enum : uint8_t { ST_LENGTH = 1, ST_STOPPED = 2, ST_DEAD_END = 3, ST_BAD_SOURCE = 4 };
enum : uint32_t { ALG_DEEPWALK = 0, ALG_PPR = 1, ALG_NODE2VEC = 2, ALG_METAPATH = 3 };
// Internal sampler codes: the public four, plus the same samplers reading an
// index (identical results, fewer dependent reads).
enum : uint32_t {
    SMP_NAIVE = 0, SMP_ALIAS = 1, SMP_ITS = 2, SMP_OREJ = 3, SMP_REJ = 4,
    SMP_LABEL_INDEX = 5,   // MetaPath with a label index
    SMP_NAIVE_ADJ = 6,     // NAIVE with the adjacency index
    SMP_OREJ_ADJ = 7,      // Node2Vec O-REJ with the adjacency index
    SMP_LABEL_FUSED = 8    // MetaPath with a label index that has fused entries (persistent schedule)
};

// Darts per O-REJ or REJ move at most (then the last dart is taken).  O-REJ:
// with every threshold >= 1 the cap is reached with probability below
// e^-256.  REJ: a dart at the row's heaviest edge always hits, so the cap is
// reached with probability (1 - sum w / (d p*))^(2^24), below e^-65536 when
// the row's weights differ by at most a factor 256.
constexpr uint32_t kMaxDarts = 1u << 24;

struct Tuning {
    uint32_t walkers_per_lane;
    uint32_t block_threads;
    uint32_t blocks_per_cu;
    uint32_t queue_chunk;
    uint32_t coop_degree;     // MetaPath scan: rows at least this long are scanned by the whole wave
    uint32_t its_gallop_degree;   // ITS: rows at least this long search from the guessed slot
    uint32_t n2v_search_degree;   // Node2Vec + edge index: prev rows at most this long are searched
    bool lds_graph;           // NAIVE DeepWalk / PPR on a graph that fits one workgroup's LDS: walk it there
};

struct DeviceInfo {
    int device;
    int num_cus;
    int lds_per_cu;     // bytes of LDS a CU holds
    int lds_per_block;  // bytes of LDS one workgroup may allocate
};

// Host launchers (tables.hip, walk.hip).  Return hipSuccess or the launch error.
hipError_t launch_alias_build(const GraphDev &g, uint4 *out, hipStream_t s);
// Small graphs (walk_small.hip): does the CSR fit one workgroup's LDS (int32
// row offsets, uint16 destinations)?  If so, persistent NAIVE DeepWalk / PPR
// walk with the graph in LDS; same results as the persistent kernel.
bool small_graph_fits(const GraphDev &g, const DeviceInfo &di);
hipError_t launch_walk_small(const GraphDev &g, const WalkDev &w, uint32_t algo, const DeviceInfo &di, void *ws,
                             hipStream_t s);
hipError_t launch_its_build(const GraphDev &g, uint64_t *prefix, uint4 *next, uint64_t *vw, hipStream_t s);
hipError_t launch_validate(const GraphDev &g, unsigned long long *d_bad, hipStream_t s);
// Counts sources outside [0, n) into *d_bad (cleared first by a kernel).
hipError_t launch_validate_sources(const int32_t *src, uint64_t nq, int32_t n, unsigned long long *d_bad,
                                   hipStream_t s);
hipError_t launch_label_index_build(const GraphDev &g, uint32_t nlab, int32_t *loff, int32_t *lcol, hipStream_t s);
hipError_t launch_label_fused_build(const GraphDev &g, uint32_t nlab, const int32_t *loff, const int32_t *lcol,
                                    uint4 *out, hipStream_t s);
hipError_t launch_adjacency_build(const GraphDev &g, uint4 *out, hipStream_t s);
hipError_t launch_edge_set_build(const GraphDev &g, unsigned long long *keys, unsigned long long slots, hipStream_t s);
hipError_t launch_symmetry_check(const GraphDev &g, unsigned long long *d_bad, hipStream_t s);
hipError_t launch_rej_build(const GraphDev &g, uint4 *records, uint32_t *pmax, hipStream_t s);

size_t walk_workspace_bytes(uint32_t mode, uint64_t nq, uint32_t max_len);
hipError_t launch_walk(const GraphDev &g, const TableDev &t, uint32_t algo, uint32_t sampler,
                       const WalkDev &w, uint32_t mode, const Tuning &tu, const DeviceInfo &di,
                       void *d_ws, size_t ws_bytes, hipStream_t s);
// PPR in the persistent schedule, counting end vertices instead of writing paths.
hipError_t launch_ppr_counts(const GraphDev &g, const TableDev &t, uint32_t sampler, const WalkDev &w,
                             const Tuning &tu, const DeviceInfo &di, void *ws, hipStream_t s);

DeviceInfo device_info();
void set_error(const std::string &msg);

// Table kinds behind a trw_table: the sampler codes for ALIAS / ITS tables,
// and two index kinds.
constexpr uint32_t kLabelIndexKind = 0x100;
constexpr uint32_t kAdjacencyKind = 0x101;
constexpr uint32_t kEdgeIndexKind = 0x102;    // adjacency records, then the edge hash set

// ITS table: the prefix (256-aligned), then the next-slot records, then W[n].
inline size_t its_prefix_bytes(int64_t m) { return ((8 * (size_t)m) + 255) / 256 * 256; }
inline size_t its_next_bytes(int64_t m) { return ((32 * (size_t)m) + 255) / 256 * 256; }

// Bytes of the slot records at the start of a REJ table (256-aligned); p*[n] follows.
inline size_t rej_records_bytes(int64_t m) { return ((32 * (size_t)m) + 255) / 256 * 256; }

// Bytes of the adjacency records at the start of an edge index (256-aligned).
inline size_t edge_index_records_bytes(int64_t m) { return ((16 * (size_t)m) + 255) / 256 * 256; }

// Accessors for the opaque handles (defined with them in abi.hip).
const GraphDev &graph_dev(trw_graph g);
bool table_view(trw_table t, uint32_t kind, const void **buf, trw_graph *graph);

}  // namespace trw
