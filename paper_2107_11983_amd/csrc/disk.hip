// Walks over a CSR graph kept in a file: the graph is split into vertex
// ranges, one range ("partition") is resident on the device at a time, and
// the queries waiting in it walk until they end or step into another range.
// The paper leaves graphs larger than memory to future work (Future
// Extension: an external-memory system hosting the graph on disk) and
// describes, among related systems, the scheme used here: load the partition
// holding the most queries, run each of its queries until it completes or
// leaves, swap, repeat (Related Work).  The moves are the batch walker's
// (same random contract, same tables, built on the device for the resident
// range at each load), so a query's path is the one trw_walk gives on the
// whole graph.
//
// Device view of a resident partition [v0, v1) with edges [e0, e1): a row
// offset array over all n + 1 vertices holding offsets relative to e0 (0 below
// v0 and e1 - e0 above v1, so rows outside the range are empty), the range's
// destinations, weights and labels, and its table.  Destinations keep their
// global ids; a walker whose vertex falls outside [v0, v1) leaves.
#include <hip/hip_runtime.h>

#include <errno.h>
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "walk_common.hpp"

struct trw_disk_graph_s {
    int fd;
    int64_t n, m;
    uint32_t flags;
    std::vector<int64_t> row_ptr;        // n + 1
    std::vector<int64_t> vstart;         // partitions + 1 vertex starts (vstart[parts] = n)
    std::vector<uint8_t> checked;        // destinations of partition i checked to lie in [0, n)
    int64_t max_edges, max_verts;        // largest partition
    uint64_t off_col, off_weight, off_label;
};

namespace trw {
namespace {

constexpr char kMagic[8] = {'T', 'R', 'W', 'C', 'S', 'R', '1', '\0'};
constexpr uint64_t kHeaderBytes = 32;
constexpr uint64_t kMaxParts = 1u << 24;

trw_status dfail(trw_status st, const std::string &m) {
    set_error(m);
    return st;
}

size_t r256(size_t x) { return (x + 255) / 256 * 256; }

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

bool read_at(int fd, void *dst, size_t bytes, uint64_t off) {
    char *p = static_cast<char *>(dst);
    while (bytes > 0) {
        const ssize_t r = pread(fd, p, bytes, (off_t)off);
        if (r < 0 && errno == EINTR) continue;
        if (r <= 0) return false;
        p += r;
        bytes -= (size_t)r;
        off += (uint64_t)r;
    }
    return true;
}

bool write_all(int fd, const void *src, size_t bytes) {
    const char *p = static_cast<const char *>(src);
    while (bytes > 0) {
        const ssize_t r = write(fd, p, bytes);
        if (r < 0 && errno == EINTR) continue;
        if (r <= 0) return false;
        p += r;
        bytes -= (size_t)r;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// A waiting walker: query index, current vertex, moves made, its partition.
struct alignas(16) DRec {
    uint32_t qi;
    int32_t cur;
    uint32_t k;
    uint32_t part;
};

// The partition holding v: the largest i with vstart[i] <= v.
__device__ __forceinline__ uint32_t part_of(const int32_t *__restrict__ vstart, uint32_t parts, int32_t v) {
    uint32_t lo = 0, hi = parts;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (vstart[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_disk_fill(uint32_t *p, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Row offsets outside the resident range: 0 below v0, mp above v1.
__global__ void k_disk_rows(int32_t *rp, int64_t n, int64_t v0, int64_t v1, int32_t mp) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
        if (v < v0) rp[v] = 0;
        else if (v > v1) rp[v] = mp;
    }
}

// Sources: a bad one ends at once; the others start a path and wait in
// their partition.
__global__ void __launch_bounds__(256) k_disk_init(WalkDev a, int32_t n, const int32_t *__restrict__ vstart,
                                                   uint32_t parts, DRec *__restrict__ out, uint32_t *count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = 0; base < a.nq; base += stride) {
        const uint64_t i = base + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        bool keep = false;
        int32_t s = 0;
        if (i < a.nq) {
            s = a.sources[i];
            if (s < 0 || s >= n) {
                a.lengths[i] = 0;
                a.status[i] = ST_BAD_SOURCE;
            } else {
                a.paths[i * a.stride] = s;
                keep = true;
            }
        }
        const uint32_t slot = wave_append(count, keep);
        if (keep) out[slot] = DRec{(uint32_t)i, s, 0u, part_of(vstart, parts, s)};
    }
}

__global__ void k_disk_hist(const DRec *__restrict__ in, const uint32_t *count, uint32_t *hist) {
    const uint32_t n = *count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        atomicAdd(&hist[in[i].part], 1u);
}

// The waiting list grouped by partition: records of partitions other than
// `skip` move, in order, to their partition's new start; the newly arrived
// ones follow them (in any order: a walk does not depend on its position).
__global__ void k_disk_move_old(const DRec *__restrict__ in, uint32_t n_in, uint32_t skip,
                                const uint32_t *__restrict__ old_off, const uint32_t *__restrict__ new_off,
                                DRec *__restrict__ out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_in; i += gridDim.x * blockDim.x) {
        const DRec r = in[i];
        if (r.part != skip) out[new_off[r.part] + (i - old_off[r.part])] = r;
    }
}

__global__ void k_disk_place_new(const DRec *__restrict__ in, const uint32_t *count, const uint32_t *__restrict__ base,
                                 uint32_t *cursor, DRec *__restrict__ out) {
    const uint32_t n = *count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const DRec r = in[i];
        out[base[r.part] + atomicAdd(&cursor[r.part], 1u)] = r;
    }
}

// One move from cur (row [off, off + d), d > 0): the next vertex, or -1 when
// the row has no eligible edge.  r holds move k's block; REJ leaves the
// hitting dart's block in it (PPR's stop coin).
template <uint32_t ALGO, uint32_t SMP>
__device__ __forceinline__ int32_t disk_move(const GraphDev &g, const TableDev &t, const WalkDev &a, uint64_t qid,
                                             uint32_t k, int32_t cur, int32_t off, uint32_t d, Rand4 &r) {
    if (ALGO == ALG_METAPATH) {
        // the edges whose label is the schema's for move k; the j-th of them
        // in row order, j = scale32(r0, their count)
        const uint32_t si = k % a.schema_len;
        const uint64_t word = si < 8 ? a.schema_lo : a.schema_hi;
        const uint8_t want = (uint8_t)(word >> ((si & 7u) * 8u));
        const uint8_t *__restrict__ lab = g.label + off;
        uint32_t cnt = 0;
        for (uint32_t i = 0; i < d; ++i) cnt += lab[i] == want;
        if (cnt == 0) return -1;
        uint32_t j = scale32(r.r0, cnt);
        for (uint32_t i = 0;; ++i) {
            if (lab[i] == want) {
                if (j == 0) return g.col[off + i];
                --j;
            }
        }
    }
    if (SMP == SMP_ALIAS) {
        const uint64_t e = (uint64_t)(uint32_t)off + scale32(r.r0, d);
        const uint4 e0 = t.alias[2 * e], e1 = t.alias[2 * e + 1];
        int32_t no, nd;
        return alias_pick(e0, e1, r.r1, no, nd);
    }
    if (SMP == SMP_REJ) {
        int32_t no, nd;
        uint32_t npm;
        return rej_move(t, a, qid, k, off, d, t.pmax[cur], r, no, nd, npm);
    }
    return static_next<SMP>(g, t, off, d, r, a.its_gallop);
}

// Every waiting walker of the resident partition [v0, v1) moves until it
// ends (its length and status written) or its vertex leaves the range (it
// is appended to `out` with its new partition).
template <uint32_t ALGO, uint32_t SMP>
__global__ void __launch_bounds__(256) k_disk_walk(GraphDev g, TableDev t, WalkDev a, int32_t v0, int32_t v1,
                                                   const DRec *__restrict__ in, uint32_t n_in,
                                                   const int32_t *__restrict__ vstart, uint32_t parts,
                                                   DRec *__restrict__ out, uint32_t *count_out) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = 0; base < n_in; base += stride) {
        const uint32_t idx = base + blockIdx.x * blockDim.x + threadIdx.x;
        bool leave = false;
        DRec rc{0u, 0, 0u, 0u};
        if (idx < n_in) {
            rc = in[idx];
            const uint64_t qid = a.qid_base + rc.qi;
            int32_t *__restrict__ path = a.paths + (uint64_t)rc.qi * a.stride;
            uint8_t st = 0;
            for (;;) {
                if (rc.cur < v0 || rc.cur >= v1) {
                    leave = true;
                    break;
                }
                const int32_t off = g.row_ptr[rc.cur];
                const uint32_t d = (uint32_t)(g.row_ptr[rc.cur + 1] - off);
                Rand4 r = philox(rc.k, 0, qid, a.seed);
                const int32_t nxt = d != 0 ? disk_move<ALGO, SMP>(g, t, a, qid, rc.k, rc.cur, off, d, r) : -1;
                if (nxt < 0) {
                    st = ST_DEAD_END;
                    break;
                }
                path[rc.k + 1] = nxt;
                ++rc.k;
                if (ALGO == ALG_PPR && r.r2 < a.stop_q32) {
                    st = ST_STOPPED;
                    break;
                }
                if (rc.k == a.max_len) {
                    st = ST_LENGTH;
                    break;
                }
                rc.cur = nxt;
            }
            if (leave) {
                rc.part = part_of(vstart, parts, rc.cur);
            } else {
                a.lengths[rc.qi] = rc.k;
                a.status[rc.qi] = st;
            }
        }
        const uint32_t slot = wave_append(count_out, leave);
        if (leave) out[slot] = rc;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
bool needs_weights(uint32_t sampler, uint32_t algo) {
    return algo != TRW_A_METAPATH && (sampler == TRW_S_ALIAS || sampler == TRW_S_ITS || sampler == TRW_S_REJ);
}

size_t table_bytes(uint32_t algo, uint32_t sampler, int64_t mp, int64_t n) {
    if (algo == TRW_A_METAPATH) return 0;
    switch (sampler) {
        case TRW_S_ALIAS: return kAliasEntryBytes * (size_t)mp;
        case TRW_S_ITS: return its_prefix_bytes(mp) + its_next_bytes(mp) + sizeof(uint64_t) * (size_t)n;
        case TRW_S_REJ: return rej_records_bytes(mp) + sizeof(uint32_t) * (size_t)n;
        default: return 0;
    }
}

// Offsets of the pieces of the device workspace and of the pinned buffer.
struct Layout {
    size_t rp, col, wgt, lab, table, lists[3], vstart, hist, cursor, new_off, old_off, base, count, dev_total;
    size_t h_rp, h_col, h_wgt, h_lab, h_hist, h_new_off, h_old_off, h_base, host_total;
};

Layout layout(const trw_disk_graph_s &g, const trw_walk_params &p, uint64_t nq) {
    const size_t parts = g.vstart.size() - 1;
    const size_t mp = (size_t)g.max_edges;
    const bool w = needs_weights(p.sampler, p.algo), l = p.algo == TRW_A_METAPATH;
    Layout L{};
    size_t o = 0;
    auto take = [&o](size_t bytes) { const size_t at = o; o += r256(bytes); return at; };
    L.rp = take(4 * ((size_t)g.n + 1));
    L.col = take(4 * mp);
    L.wgt = take(w ? 4 * mp : 0);
    L.lab = take(l ? mp : 0);
    L.table = take(table_bytes(p.algo, p.sampler, (int64_t)mp, g.n));
    for (auto &x : L.lists) x = take(sizeof(DRec) * (size_t)nq);
    L.vstart = take(4 * (parts + 1));
    L.hist = take(4 * parts);
    L.cursor = take(4 * parts);
    L.new_off = take(4 * parts);
    L.old_off = take(4 * parts);
    L.base = take(4 * parts);
    L.count = take(4);
    L.dev_total = o;
    o = 0;
    L.h_rp = take(4 * ((size_t)g.max_verts + 1));
    L.h_col = take(4 * mp);
    L.h_wgt = take(w ? 4 * mp : 0);
    L.h_lab = take(l ? mp : 0);
    L.h_hist = take(4 * parts + 4);
    L.h_new_off = take(4 * parts);
    L.h_old_off = take(4 * parts);
    L.h_base = take(4 * parts);
    L.host_total = o;
    return L;
}

trw_status check_walk(const trw_disk_graph_s *g, const trw_walk_params *p) {
    if (!g) return dfail(TRW_E_INVALID, "disk graph is NULL");
    if (!p) return dfail(TRW_E_INVALID, "params is NULL");
    if (p->algo == TRW_A_NODE2VEC)
        return dfail(TRW_E_UNSUPPORTED, "Node2Vec reads the previous vertex's row, which may lie in another partition");
    if (p->algo == TRW_A_DEEPWALK || p->algo == TRW_A_PPR) {
        if (p->sampler != TRW_S_NAIVE && p->sampler != TRW_S_ALIAS && p->sampler != TRW_S_ITS &&
            p->sampler != TRW_S_REJ)
            return dfail(TRW_E_UNSUPPORTED, "sampler not provided for this algorithm");
    } else if (p->algo == TRW_A_METAPATH) {
        if (p->sampler != TRW_S_ITS) return dfail(TRW_E_UNSUPPORTED, "MetaPath walks with ITS");
        if (p->schema_len == 0 || p->schema_len > 16) return dfail(TRW_E_INVALID, "schema_len must be in 1..16");
        if (!(g->flags & TRW_DISK_LABELS)) return dfail(TRW_E_INVALID, "MetaPath needs edge labels");
    } else {
        return dfail(TRW_E_UNSUPPORTED, "unknown algorithm");
    }
    if (p->max_len == 0 || p->max_len > 65535) return dfail(TRW_E_INVALID, "max_len must be in 1..65535");
    if (needs_weights(p->sampler, p->algo) && !(g->flags & TRW_DISK_WEIGHTS))
        return dfail(TRW_E_INVALID, "ALIAS / ITS / REJ walks need edge weights");
    return TRW_OK;
}

template <uint32_t ALGO, uint32_t SMP>
void launch_disk_walk(const GraphDev &g, const TableDev &t, const WalkDev &w, int32_t v0, int32_t v1,
                      const DRec *in, uint32_t n_in, const int32_t *vstart, uint32_t parts, DRec *out,
                      uint32_t *count, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_disk_walk<ALGO, SMP>), dim3(blocks), dim3(256), 0, s, g, t, w, v0, v1, in, n_in, vstart,
                       parts, out, count);
}

template <uint32_t ALGO>
void dispatch_walk(uint32_t sampler, const GraphDev &g, const TableDev &t, const WalkDev &w, int32_t v0, int32_t v1,
                   const DRec *in, uint32_t n_in, const int32_t *vstart, uint32_t parts, DRec *out,
                   uint32_t *count, uint32_t blocks, hipStream_t s) {
    switch (sampler) {
        case TRW_S_NAIVE:
            launch_disk_walk<ALGO, SMP_NAIVE>(g, t, w, v0, v1, in, n_in, vstart, parts, out, count, blocks, s);
            break;
        case TRW_S_ALIAS:
            launch_disk_walk<ALGO, SMP_ALIAS>(g, t, w, v0, v1, in, n_in, vstart, parts, out, count, blocks, s);
            break;
        case TRW_S_REJ:
            launch_disk_walk<ALGO, SMP_REJ>(g, t, w, v0, v1, in, n_in, vstart, parts, out, count, blocks, s);
            break;
        default:
            launch_disk_walk<ALGO, SMP_ITS>(g, t, w, v0, v1, in, n_in, vstart, parts, out, count, blocks, s);
    }
}

uint32_t grid_for(uint64_t items, const DeviceInfo &di) {
    const uint64_t want = (items + 255) / 256;
    const uint64_t cap = (uint64_t)di.num_cus * 8;
    return (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
}

}  // namespace
}  // namespace trw

using namespace trw;

extern "C" {

trw_status trw_disk_graph_write(const char *path, int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                                const uint32_t *weight, const uint8_t *label) {
    if (!path || !row_ptr || (m > 0 && !col)) return dfail(TRW_E_INVALID, "path / row_ptr / col is NULL");
    if (n < 1 || n >= (int64_t(1) << 31) || m < 0) return dfail(TRW_E_INVALID, "n must be in 1..2^31-1, m >= 0");
    const int fd = open(path, O_WRONLY | O_CREAT | O_TRUNC, 0644);
    if (fd < 0) return dfail(TRW_E_INVALID, std::string("cannot create ") + path + ": " + strerror(errno));
    const uint64_t head[3] = {(uint64_t)n, (uint64_t)m,
                              (uint64_t)((weight ? TRW_DISK_WEIGHTS : 0) | (label ? TRW_DISK_LABELS : 0))};
    bool ok = write_all(fd, kMagic, 8) && write_all(fd, head, sizeof(head)) &&
              write_all(fd, row_ptr, sizeof(int64_t) * ((size_t)n + 1)) &&
              (m == 0 || write_all(fd, col, sizeof(int32_t) * (size_t)m)) &&
              (!weight || m == 0 || write_all(fd, weight, sizeof(uint32_t) * (size_t)m)) &&
              (!label || m == 0 || write_all(fd, label, (size_t)m));
    ok = (close(fd) == 0) && ok;
    if (!ok) return dfail(TRW_E_INVALID, std::string("write to ") + path + " failed");
    return TRW_OK;
}

trw_status trw_disk_graph_open(const char *path, uint64_t part_edges, trw_disk_graph *out) {
    if (!path || !out) return dfail(TRW_E_INVALID, "path / out is NULL");
    if (part_edges >= (uint64_t(1) << 31)) return dfail(TRW_E_INVALID, "part_edges must be < 2^31");
    if (part_edges == 0) part_edges = (uint64_t(1) << 31) - 1;
    const int fd = open(path, O_RDONLY);
    if (fd < 0) return dfail(TRW_E_INVALID, std::string("cannot open ") + path + ": " + strerror(errno));
    auto bad = [fd](const std::string &m) {
        close(fd);
        return dfail(TRW_E_INVALID, m);
    };
    char magic[8];
    uint64_t head[3];
    if (!read_at(fd, magic, 8, 0) || !read_at(fd, head, sizeof(head), 8)) return bad("file shorter than its header");
    if (std::memcmp(magic, kMagic, 8) != 0) return bad("not a CSR file (bad magic)");
    const uint64_t n = head[0], m = head[1], flags = head[2];
    if (n < 1 || n >= (uint64_t(1) << 31)) return bad("n must be in 1..2^31-1");
    if (m >= (uint64_t(1) << 62) || (flags & ~uint64_t(3))) return bad("bad m or flags");
    const uint64_t off_col = kHeaderBytes + 8 * (n + 1);
    const uint64_t off_weight = off_col + 4 * m;
    const uint64_t off_label = off_weight + ((flags & TRW_DISK_WEIGHTS) ? 4 * m : 0);
    const uint64_t total = off_label + ((flags & TRW_DISK_LABELS) ? m : 0);
    struct stat sb;
    if (fstat(fd, &sb) != 0 || (uint64_t)sb.st_size != total) return bad("file size does not match its header");
    auto *g = new (std::nothrow) trw_disk_graph_s{};
    if (!g) return bad("out of host memory");
    try {
        g->row_ptr.resize(n + 1);
    } catch (...) {
        delete g;
        return bad("out of host memory for row_ptr");
    }
    if (!read_at(fd, g->row_ptr.data(), 8 * (n + 1), kHeaderBytes)) {
        delete g;
        return bad("cannot read row_ptr");
    }
    const auto &rp = g->row_ptr;
    if (rp[0] != 0 || rp[n] != (int64_t)m) {
        delete g;
        return bad("row_ptr must start at 0 and end at m");
    }
    for (uint64_t v = 0; v < n; ++v) {
        const int64_t d = rp[v + 1] - rp[v];
        if (d < 0 || d >= (int64_t(1) << 31)) {
            delete g;
            return bad("row " + std::to_string(v) + " has a negative length or 2^31 edges or more");
        }
    }
    // vertex ranges of at most part_edges edges; a longer row alone
    g->vstart.push_back(0);
    int64_t max_e = 0, max_v = 0;
    for (int64_t v = 0; v < (int64_t)n;) {
        const int64_t v0 = v, e0 = rp[v];
        ++v;
        while (v < (int64_t)n && rp[v + 1] - e0 <= (int64_t)part_edges) ++v;
        g->vstart.push_back(v);
        max_e = std::max(max_e, rp[v] - e0);
        max_v = std::max(max_v, v - v0);
        if (g->vstart.size() - 1 > kMaxParts) {
            delete g;
            return bad("more than 2^24 partitions: part_edges too small");
        }
    }
    g->fd = fd;
    g->n = (int64_t)n;
    g->m = (int64_t)m;
    g->flags = (uint32_t)flags;
    g->checked.assign(g->vstart.size() - 1, 0);
    g->max_edges = max_e;
    g->max_verts = max_v;
    g->off_col = off_col;
    g->off_weight = off_weight;
    g->off_label = off_label;
    *out = g;
    return TRW_OK;
}

trw_status trw_disk_graph_info(trw_disk_graph g, uint64_t *n, uint64_t *m, uint32_t *flags, uint32_t *parts) {
    if (!g) return dfail(TRW_E_INVALID, "disk graph is NULL");
    if (n) *n = (uint64_t)g->n;
    if (m) *m = (uint64_t)g->m;
    if (flags) *flags = g->flags;
    if (parts) *parts = (uint32_t)(g->vstart.size() - 1);
    return TRW_OK;
}

trw_status trw_disk_graph_partition(trw_disk_graph g, uint32_t i, int64_t *v_begin, int64_t *v_end, int64_t *e_begin,
                                    int64_t *e_end) {
    if (!g) return dfail(TRW_E_INVALID, "disk graph is NULL");
    if ((size_t)i + 1 >= g->vstart.size()) return dfail(TRW_E_INVALID, "partition index out of range");
    const int64_t v0 = g->vstart[i], v1 = g->vstart[i + 1];
    if (v_begin) *v_begin = v0;
    if (v_end) *v_end = v1;
    if (e_begin) *e_begin = g->row_ptr[v0];
    if (e_end) *e_end = g->row_ptr[v1];
    return TRW_OK;
}

trw_status trw_disk_graph_close(trw_disk_graph g) {
    if (!g) return dfail(TRW_E_INVALID, "disk graph is NULL");
    close(g->fd);
    delete g;
    return TRW_OK;
}

trw_status trw_disk_walk_bytes(trw_disk_graph g, const trw_walk_params *p, uint64_t nq, size_t *device_bytes,
                               size_t *host_bytes) {
    trw_status st = check_walk(g, p);
    if (st != TRW_OK) return st;
    if (!device_bytes || !host_bytes) return dfail(TRW_E_INVALID, "device_bytes / host_bytes is NULL");
    if (nq >= (uint64_t(1) << 32)) return dfail(TRW_E_INVALID, "nq must be < 2^32");
    const Layout L = layout(*g, *p, nq);
    *device_bytes = L.dev_total;
    *host_bytes = L.host_total;
    return TRW_OK;
}

trw_status trw_disk_walk(trw_disk_graph g, const trw_walk_params *p, const int32_t *d_sources, uint64_t nq,
                         uint64_t qid_base, int32_t *d_paths, uint64_t path_stride, uint32_t *d_lengths,
                         uint8_t *d_status, void *d_ws, size_t ws_bytes, void *h_pinned, size_t h_bytes,
                         trw_disk_walk_stats *stats, trw_stream_t stream) {
    const uint64_t t_start = now_ns();
    trw_status st = check_walk(g, p);
    if (st != TRW_OK) return st;
    if (nq >= (uint64_t(1) << 32)) return dfail(TRW_E_INVALID, "nq must be < 2^32");
    if (path_stride < (uint64_t)p->max_len + 1) return dfail(TRW_E_INVALID, "path_stride < max_len + 1");
    trw_disk_walk_stats S{};
    if (nq == 0) {
        if (stats) *stats = S;
        return TRW_OK;
    }
    if (!d_sources || !d_paths || !d_lengths || !d_status)
        return dfail(TRW_E_INVALID, "sources / paths / lengths / status is NULL");
    const Layout L = layout(*g, *p, nq);
    if (!d_ws || ws_bytes < L.dev_total || (reinterpret_cast<uintptr_t>(d_ws) & 255))
        return dfail(TRW_E_INVALID, "workspace NULL, too small or not 256-byte aligned");
    if (!h_pinned || h_bytes < L.host_total || (reinterpret_cast<uintptr_t>(h_pinned) & 255))
        return dfail(TRW_E_INVALID, "pinned buffer NULL, too small or not 256-byte aligned");

    auto s = static_cast<hipStream_t>(stream);
    char *D = static_cast<char *>(d_ws);
    char *H = static_cast<char *>(h_pinned);
    const uint32_t parts = (uint32_t)(g->vstart.size() - 1);
    const bool want_w = needs_weights(p->sampler, p->algo), want_l = p->algo == TRW_A_METAPATH;
    const DeviceInfo di = device_info();

    int32_t *d_rp = reinterpret_cast<int32_t *>(D + L.rp);
    int32_t *d_col = reinterpret_cast<int32_t *>(D + L.col);
    uint32_t *d_wgt = want_w ? reinterpret_cast<uint32_t *>(D + L.wgt) : nullptr;
    uint8_t *d_lab = want_l ? reinterpret_cast<uint8_t *>(D + L.lab) : nullptr;
    char *d_tab = D + L.table;
    DRec *lists[3] = {reinterpret_cast<DRec *>(D + L.lists[0]), reinterpret_cast<DRec *>(D + L.lists[1]),
                      reinterpret_cast<DRec *>(D + L.lists[2])};
    int32_t *d_vstart = reinterpret_cast<int32_t *>(D + L.vstart);
    uint32_t *d_hist = reinterpret_cast<uint32_t *>(D + L.hist);
    uint32_t *d_cursor = reinterpret_cast<uint32_t *>(D + L.cursor);
    uint32_t *d_new_off = reinterpret_cast<uint32_t *>(D + L.new_off);
    uint32_t *d_old_off = reinterpret_cast<uint32_t *>(D + L.old_off);
    uint32_t *d_base = reinterpret_cast<uint32_t *>(D + L.base);
    uint32_t *d_count = reinterpret_cast<uint32_t *>(D + L.count);
    int32_t *h_rp = reinterpret_cast<int32_t *>(H + L.h_rp);
    int32_t *h_col = reinterpret_cast<int32_t *>(H + L.h_col);
    uint32_t *h_wgt = reinterpret_cast<uint32_t *>(H + L.h_wgt);
    uint8_t *h_lab = reinterpret_cast<uint8_t *>(H + L.h_lab);
    uint32_t *h_hist = reinterpret_cast<uint32_t *>(H + L.h_hist);   // parts counts, then the arrival count
    uint32_t *h_new_off = reinterpret_cast<uint32_t *>(H + L.h_new_off);
    uint32_t *h_old_off = reinterpret_cast<uint32_t *>(H + L.h_old_off);
    uint32_t *h_base = reinterpret_cast<uint32_t *>(H + L.h_base);

    WalkDev w{};
    w.max_len = p->max_len;
    w.stop_q32 = p->algo == TRW_A_PPR ? p->stop_q32 : 0;
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
    w.its_gallop = 1;

    hipError_t e = hipSuccess;
    auto device_error = [&](const char *what) {
        (void)hipStreamSynchronize(s);
        return dfail(TRW_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    auto host_error = [&](const std::string &what) {
        (void)hipStreamSynchronize(s);   // nothing of this call runs on after it returns
        return dfail(TRW_E_INVALID, what);
    };
    auto fill = [&](uint32_t *ptr, uint32_t count, uint32_t v) {
        if (count) hipLaunchKernelGGL(k_disk_fill, dim3((count + 255) / 256), dim3(256), 0, s, ptr, count, v);
    };
    // histogram of the arrivals in lists[2] (count in d_count) into h_hist; waits
    auto read_arrivals = [&]() {
        fill(d_hist, parts, 0u);
        hipLaunchKernelGGL(k_disk_hist, dim3(grid_for(nq, di)), dim3(256), 0, s, lists[2], d_count, d_hist);
        e = hipMemcpyAsync(h_hist, d_hist, 4 * (size_t)parts, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h_hist + parts, d_count, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e == hipSuccess;
    };

    // partition starts on the device (int32: n < 2^31)
    {
        std::vector<int32_t> vs(g->vstart.begin(), g->vstart.end());
        e = hipMemcpyAsync(d_vstart, vs.data(), 4 * vs.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return device_error("partition starts upload");
    }
    // the sources wait in their partitions
    fill(d_count, 1, 0u);
    hipLaunchKernelGGL(k_disk_init, dim3(grid_for(nq, di)), dim3(256), 0, s, w, (int32_t)g->n, d_vstart, parts,
                       lists[2], d_count);
    e = hipGetLastError();
    if (e != hipSuccess || !read_arrivals()) return device_error("start");

    // host copies of the waiting list's layout: per partition its count and start
    std::vector<uint64_t> counts(parts, 0), next(parts, 0), off(parts, 0);
    DRec *cur = lists[0], *spare = lists[1];
    int64_t resident = -1;
    uint32_t skip = 0xFFFFFFFFu;   // the partition just walked (its old records are consumed)
    uint64_t old_total = 0;
    for (;;) {
        // regroup into `spare`: each partition's old records (none for `skip`),
        // then its arrivals.  The pinned offset arrays are written here only,
        // after the previous iteration's wait, and read by this one's copies.
        uint64_t acc = 0;
        for (uint32_t q = 0; q < parts; ++q) {
            const uint64_t kept = q == skip ? 0 : counts[q];
            next[q] = kept + h_hist[q];
            h_old_off[q] = (uint32_t)off[q];
            h_new_off[q] = (uint32_t)acc;
            h_base[q] = (uint32_t)(acc + kept);
            acc += next[q];
        }
        const uint64_t waiting = acc;
        const uint64_t old_kept = old_total - (skip == 0xFFFFFFFFu ? 0 : counts[skip]);
        e = hipMemcpyAsync(d_new_off, h_new_off, 4 * (size_t)parts, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_base, h_base, 4 * (size_t)parts, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && old_kept > 0)
            e = hipMemcpyAsync(d_old_off, h_old_off, 4 * (size_t)parts, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return device_error("offsets upload");
        if (old_kept > 0)
            hipLaunchKernelGGL(k_disk_move_old, dim3(grid_for(old_total, di)), dim3(256), 0, s, cur,
                               (uint32_t)old_total, skip, d_old_off, d_new_off, spare);
        fill(d_cursor, parts, 0u);
        hipLaunchKernelGGL(k_disk_place_new, dim3(grid_for(h_hist[parts], di)), dim3(256), 0, s, lists[2], d_count,
                           d_base, d_cursor, spare);
        e = hipGetLastError();
        if (e != hipSuccess) return device_error("regroup launch");
        std::swap(cur, spare);
        counts.swap(next);
        for (uint32_t q = 0; q < parts; ++q) off[q] = h_new_off[q];
        old_total = waiting;
        if (waiting == 0) break;

        // the partition with the most waiting queries (the lowest index among equals)
        uint32_t pbest = 0;
        for (uint32_t q = 1; q < parts; ++q)
            if (counts[q] > counts[pbest]) pbest = q;
        const int64_t v0 = g->vstart[pbest], v1 = g->vstart[pbest + 1];
        const int64_t e0 = g->row_ptr[v0], e1 = g->row_ptr[v1];
        const int64_t mp = e1 - e0;
        GraphDev view{d_rp, d_col, d_wgt, d_lab, (int32_t)g->n, (int32_t)mp, 0};
        TableDev t{};
        if (p->algo != TRW_A_METAPATH && p->sampler == TRW_S_ALIAS) {
            t.alias = reinterpret_cast<const uint4 *>(d_tab);
        } else if (p->algo != TRW_A_METAPATH && p->sampler == TRW_S_REJ) {
            t.rej = reinterpret_cast<const uint4 *>(d_tab);
            t.pmax = reinterpret_cast<const uint32_t *>(d_tab + rej_records_bytes(mp));
        } else if (p->algo != TRW_A_METAPATH && p->sampler == TRW_S_ITS) {
            t.prefix = reinterpret_cast<const uint64_t *>(d_tab);
            t.its_next = reinterpret_cast<const uint4 *>(d_tab + its_prefix_bytes(mp));
            t.its_w = reinterpret_cast<const uint64_t *>(d_tab + its_prefix_bytes(mp) + its_next_bytes(mp));
        }
        if (resident != (int64_t)pbest) {
            // read the range's rows and edges, copy them, build its table
            const uint64_t t0 = now_ns();
            for (int64_t v = v0; v <= v1; ++v) h_rp[v - v0] = (int32_t)(g->row_ptr[v] - e0);
            bool ok = mp == 0 || read_at(g->fd, h_col, 4 * (size_t)mp, g->off_col + 4 * (uint64_t)e0);
            if (ok && want_w && mp > 0) ok = read_at(g->fd, h_wgt, 4 * (size_t)mp, g->off_weight + 4 * (uint64_t)e0);
            if (ok && want_l && mp > 0) ok = read_at(g->fd, h_lab, (size_t)mp, g->off_label + (uint64_t)e0);
            S.read_ns += now_ns() - t0;
            if (!ok) return host_error("cannot read partition " + std::to_string(pbest) + " of the file");
            S.bytes_read += (uint64_t)mp * (4 + (want_w ? 4 : 0) + (want_l ? 1 : 0));
            if (!g->checked[pbest]) {
                for (int64_t i = 0; i < mp; ++i)
                    if ((uint32_t)h_col[i] >= (uint32_t)g->n)
                        return host_error("edge " + std::to_string(e0 + i) + " has a destination outside [0, n)");
                g->checked[pbest] = 1;
            }
            resident = -1;
            hipLaunchKernelGGL(k_disk_rows, dim3(grid_for((uint64_t)g->n + 1, di)), dim3(256), 0, s, d_rp, g->n, v0,
                               v1, (int32_t)mp);
            e = hipMemcpyAsync(d_rp + v0, h_rp, 4 * (size_t)(v1 - v0 + 1), hipMemcpyHostToDevice, s);
            if (e == hipSuccess && mp > 0) e = hipMemcpyAsync(d_col, h_col, 4 * (size_t)mp, hipMemcpyHostToDevice, s);
            if (e == hipSuccess && want_w && mp > 0)
                e = hipMemcpyAsync(d_wgt, h_wgt, 4 * (size_t)mp, hipMemcpyHostToDevice, s);
            if (e == hipSuccess && want_l && mp > 0)
                e = hipMemcpyAsync(d_lab, h_lab, (size_t)mp, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return device_error("partition copy");
            if (mp > 0 && p->algo != TRW_A_METAPATH) {
                if (p->sampler == TRW_S_ALIAS)
                    e = launch_alias_build(view, reinterpret_cast<uint4 *>(d_tab), s);
                else if (p->sampler == TRW_S_ITS)
                    e = launch_its_build(view, reinterpret_cast<uint64_t *>(d_tab),
                                         reinterpret_cast<uint4 *>(d_tab + its_prefix_bytes(mp)),
                                         reinterpret_cast<uint64_t *>(d_tab + its_prefix_bytes(mp) + its_next_bytes(mp)),
                                         s);
                else if (p->sampler == TRW_S_REJ)
                    e = launch_rej_build(view, reinterpret_cast<uint4 *>(d_tab),
                                         reinterpret_cast<uint32_t *>(d_tab + rej_records_bytes(mp)), s);
                if (e != hipSuccess) return device_error("table build launch");
            }
            resident = pbest;
            ++S.loads;
        }
        // walk every query waiting there; those that leave arrive in lists[2].
        // Each walker of a run moves at least once or ends, so there are at most
        // nq * max_len runs with work.
        if (++S.runs > nq * (uint64_t)p->max_len) return host_error("partition walks made no progress");
        fill(d_count, 1, 0u);
        const uint32_t n_in = (uint32_t)counts[pbest];
        const DRec *in = cur + off[pbest];
        const uint32_t blocks = grid_for(n_in, di);
        switch (p->algo) {
            case TRW_A_DEEPWALK:
                dispatch_walk<ALG_DEEPWALK>(p->sampler, view, t, w, (int32_t)v0, (int32_t)v1, in, n_in, d_vstart, parts,
                                            lists[2], d_count, blocks, s);
                break;
            case TRW_A_PPR:
                dispatch_walk<ALG_PPR>(p->sampler, view, t, w, (int32_t)v0, (int32_t)v1, in, n_in, d_vstart, parts,
                                       lists[2], d_count, blocks, s);
                break;
            default:
                launch_disk_walk<ALG_METAPATH, SMP_ITS>(view, t, w, (int32_t)v0, (int32_t)v1, in, n_in, d_vstart, parts,
                                                        lists[2], d_count, blocks, s);
        }
        e = hipGetLastError();
        if (e != hipSuccess || !read_arrivals()) return device_error("partition walk");
        skip = pbest;
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error("finish");
    S.total_ns = now_ns() - t_start;
    if (stats) *stats = S;
    return TRW_OK;
}

}  // extern "C"
