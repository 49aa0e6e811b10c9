// Walks over a CSR graph kept in a file.  The graph is split into vertex
// ranges ("partitions"); up to `slots` of them are resident on the device at
// once, and the queries waiting in resident partitions walk until they end
// or step into a partition that is not resident.  The paper leaves graphs
// larger than memory to future work (Future Extension: an external-memory
// system hosting the graph on disk) and describes, among related systems,
// the scheme used here: load the partition holding the most queries, run
// each of its queries until it completes or leaves, swap, repeat (Related
// Work).  Here HBM holds many partitions at once, so a walk crosses freely
// between resident ones and a partition is read again only after eviction.
// The moves are the batch walker's (same random contract, same tables,
// built on the device for each partition at its load), so a query's path is
// the one trw_walk gives on the whole graph.
//
// A slot holds one partition [v0, v1) with edges [e0, e1): a row offset
// array over all n + 1 vertices with offsets relative to e0 (0 below v0 and
// e1 - e0 above v1, so rows outside the range are empty), the range's
// destinations, weights and labels, and its table, built for the range's
// rows only.  Destinations keep their global ids; a per-vertex map gives the
// slot of each vertex's partition (kNoSlot when it is not resident).  A table
// record's copy of its destination's row or bound is right only for a
// destination in the same range, so a move here reads the current vertex's
// row offsets and bound itself.
#include <hip/hip_runtime.h>

#include <errno.h>
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "table_range.hpp"
#include "walk_common.hpp"

struct trw_disk_graph_s {
    int fd;
    int64_t n, m;
    uint32_t flags;
    std::vector<int64_t> row_ptr;        // n + 1
    std::vector<int64_t> vstart;         // partitions + 1 vertex starts (vstart[parts] = n)
    std::vector<uint8_t> checked;        // destinations of partition i checked to lie in [0, n)
    std::vector<uint8_t> sorted;         // rows of partition i: 0 not checked, 1 sorted, 2 not sorted
    int64_t max_edges, max_verts;        // largest partition
    uint64_t off_col, off_weight, off_label;
};

namespace trw {
namespace {

constexpr char kMagic[8] = {'T', 'R', 'W', 'C', 'S', 'R', '1', '\0'};
constexpr uint64_t kHeaderBytes = 32;
constexpr uint64_t kMaxParts = 1u << 24;
constexpr uint32_t kMaxSlots = 4096;
constexpr uint16_t kNoSlot = 0xFFFF;
constexpr size_t kReadChunk = size_t(64) << 20;   // file bytes per read (then copied while the next is read)
constexpr size_t kReadPiece = size_t(8) << 20;    // bytes per reading thread
constexpr uint32_t kLdsParts = 4096;              // keys the regroup kernels count in LDS
constexpr uint64_t kMaxPairParts = 1024;          // Node2Vec: partitions (so at most 2^20 pair keys)

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

// pread of one range split over up to 8 threads (page-cache copies and device
// queues both gain from several reads in flight).
bool read_parallel(int fd, void *dst, size_t bytes, uint64_t off) {
    const size_t pieces = std::min<size_t>(8, (bytes + kReadPiece - 1) / kReadPiece);
    if (pieces <= 1) return read_at(fd, dst, bytes, off);
    const size_t each = (bytes + pieces - 1) / pieces;
    std::atomic<bool> ok{true};
    std::vector<std::thread> th;
    th.reserve(pieces);
    for (size_t i = 0; i < pieces; ++i) {
        const size_t a = i * each, b = std::min(bytes, a + each);
        if (a >= b) break;
        auto piece = [&ok, fd, dst, off, a, b] {
            if (!read_at(fd, static_cast<char *>(dst) + a, b - a, off + a)) ok = false;
        };
        try {
            th.emplace_back(piece);
        } catch (...) {   // no thread to be had: read this piece here
            piece();
        }
    }
    for (auto &t : th) t.join();
    return ok;
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
// A waiting walker: query index, current vertex, moves made, the key it
// waits under (its partition; for Node2Vec the pair of its current and
// previous vertices' partitions, current * parts + previous), and the
// previous vertex (Node2Vec; -1 before the first move).
struct alignas(16) DRec {
    uint32_t qi;
    int32_t cur;
    uint32_t k;
    uint32_t part;
    int32_t prev;
    uint32_t pad[3];
};

// Where the pieces of a slot sit: slot s starts at base + s * stride; the
// table's parts are at fixed offsets sized for the largest partition.
struct SlotsDev {
    char *base;
    uint64_t stride;
    uint64_t o_rp, o_col, o_wgt, o_lab, o_tab;
    uint64_t tab_o1, tab_o2;   // REJ: p* at o1; ITS: next-slot records at o1, W at o2
    int32_t n;
    uint32_t has_wgt, has_lab;
};

__device__ __forceinline__ void slot_views(const SlotsDev &S, uint32_t slot, GraphDev &g, TableDev &t,
                                           uint32_t sampler) {
    char *b = S.base + (uint64_t)slot * S.stride;
    g.row_ptr = reinterpret_cast<const int32_t *>(b + S.o_rp);
    g.col = reinterpret_cast<const int32_t *>(b + S.o_col);
    g.weight = S.has_wgt ? reinterpret_cast<const uint32_t *>(b + S.o_wgt) : nullptr;
    g.label = S.has_lab ? reinterpret_cast<const uint8_t *>(b + S.o_lab) : nullptr;
    g.n = S.n;
    g.m = 0;
    g.symmetric = 0;
    char *tb = b + S.o_tab;
    if (sampler == SMP_ALIAS) {
        t.alias = reinterpret_cast<const uint4 *>(tb);
    } else if (sampler == SMP_REJ) {
        t.rej = reinterpret_cast<const uint4 *>(tb);
        t.pmax = reinterpret_cast<const uint32_t *>(tb + S.tab_o1);
    } else if (sampler == SMP_ITS) {
        t.prefix = reinterpret_cast<const uint64_t *>(tb);
    }
}

// The partition holding v: the largest i with vstart[i] <= v.
__device__ __forceinline__ uint32_t part_of(const int32_t *__restrict__ vstart, uint32_t parts, int32_t v) {
    uint32_t lo = 0, hi = parts;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (vstart[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// Lanes holding the same key share one atomic: the wave serves one key at a
// time (the number of distinct keys among its lanes).  Returns this lane's
// position among the additions to counters[key] (undefined when !active).
__device__ __forceinline__ uint32_t wave_add_by_key(uint32_t *counters, uint32_t key, bool active) {
    uint64_t todo = __ballot(active);
    uint32_t pos = 0;
    while (todo) {
        const int leader = (int)__builtin_ctzll(todo);
        const uint32_t k = __shfl(key, leader);
        const uint64_t same = __ballot(active && key == k) & todo;
        uint32_t base = 0;
        if (lane_id() == (uint32_t)leader) base = atomicAdd(&counters[k], (uint32_t)__popcll(same));
        base = __shfl(base, leader);
        if ((same >> lane_id()) & 1) pos = base + rank_below(same);
        todo &= ~same;
    }
    return pos;
}

__global__ void k_disk_fill(uint32_t *p, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Slot map entries of the vertices [lo, hi).
__global__ void k_disk_set_slot(uint16_t *vslot, int64_t lo, int64_t hi, uint16_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += stride) vslot[i] = v;
}

// Row offsets outside the slot's range: 0 below v0, mp above v1.
__global__ void k_disk_rows(int32_t *rp, int64_t n, int64_t v0, int64_t v1, int32_t mp) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
        if (v < v0) rp[v] = 0;
        else if (v > v1) rp[v] = mp;
    }
}

// Sources: a bad one ends at once; the others start a path and wait in
// their partition (pairs: under the pair (partition, partition)).
__global__ void __launch_bounds__(256) k_disk_init(WalkDev a, int32_t n, const int32_t *__restrict__ vstart,
                                                   uint32_t parts, uint32_t pairs, DRec *__restrict__ out,
                                                   uint32_t *count) {
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
        if (keep) {
            const uint32_t ps = part_of(vstart, parts, s);
            out[slot] = DRec{(uint32_t)i, s, 0u, pairs ? ps * parts + ps : ps, -1, {0u, 0u, 0u}};
        }
    }
}

// Arrivals per partition.  Up to kLdsParts partitions a workgroup counts its
// share in LDS and adds each nonzero count to memory once (a batch's walkers
// spread over few partitions would otherwise queue on few counters); beyond
// that, lanes with the same partition share one atomic per wave.
__global__ void __launch_bounds__(256) k_disk_hist(const DRec *__restrict__ in, const uint32_t *count,
                                                   uint32_t *hist, uint32_t parts) {
    extern __shared__ uint32_t sh_cnt[];
    const uint32_t n = *count;
    const uint32_t stride = gridDim.x * blockDim.x;
    const bool lds = parts <= kLdsParts;
    if (lds) {
        for (uint32_t q = threadIdx.x; q < parts; q += blockDim.x) sh_cnt[q] = 0;
        __syncthreads();
    }
    for (uint32_t base = 0; base < n; base += stride) {
        const uint32_t i = base + blockIdx.x * blockDim.x + threadIdx.x;
        const bool act = i < n;
        const uint32_t part = act ? in[i].part : 0u;
        if (lds) {
            if (act) atomicAdd(&sh_cnt[part], 1u);
        } else {
            (void)wave_add_by_key(hist, part, act);
        }
    }
    if (lds) {
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < parts; q += blockDim.x)
            if (sh_cnt[q]) atomicAdd(&hist[q], sh_cnt[q]);
    }
}

// The waiting list grouped by partition: records of partitions not walked
// (consumed[part] == 0) move, in order, to their partition's new start; the
// newly arrived ones follow them (in any order: a walk does not depend on
// its position).
__global__ void k_disk_move_old(const DRec *__restrict__ in, uint32_t n_in, const uint8_t *__restrict__ consumed,
                                const uint32_t *__restrict__ old_off, const uint32_t *__restrict__ new_off,
                                DRec *__restrict__ out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_in; i += gridDim.x * blockDim.x) {
        const DRec r = in[i];
        if (!consumed[r.part]) out[new_off[r.part] + (i - old_off[r.part])] = r;
    }
}

// Arrivals to their places after base[part].  Up to kLdsParts partitions a
// workgroup counts its share in LDS, reserves one range per partition with
// one atomic, and places its records by LDS ranks; beyond that, per wave as
// in k_disk_hist.  Launched with the same grid as the count it follows.
__global__ void __launch_bounds__(256) k_disk_place_new(const DRec *__restrict__ in, const uint32_t *count,
                                                        const uint32_t *__restrict__ base, uint32_t *cursor,
                                                        DRec *__restrict__ out, uint32_t parts) {
    extern __shared__ uint32_t sh_place[];   // counts[parts], then starts[parts]
    const uint32_t n = *count;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (parts <= kLdsParts) {
        uint32_t *cnt = sh_place, *start = sh_place + parts;
        for (uint32_t q = threadIdx.x; q < parts; q += blockDim.x) cnt[q] = 0;
        __syncthreads();
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) atomicAdd(&cnt[in[i].part], 1u);
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < parts; q += blockDim.x) {
            const uint32_t c = cnt[q];
            start[q] = c ? atomicAdd(&cursor[q], c) : 0u;
            cnt[q] = 0;
        }
        __syncthreads();
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            const DRec r = in[i];
            out[base[r.part] + start[r.part] + atomicAdd(&cnt[r.part], 1u)] = r;
        }
        return;
    }
    for (uint32_t b = 0; b < n; b += stride) {
        const uint32_t i = b + blockIdx.x * blockDim.x + threadIdx.x;
        const bool act = i < n;
        DRec r{0u, 0, 0u, 0u, -1, {0u, 0u, 0u}};
        if (act) r = in[i];
        const uint32_t pos = wave_add_by_key(cursor, r.part, act);
        if (act) out[base[r.part] + pos] = r;
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

// Every waiting walker of one resident partition moves until it ends (its
// length and status written) or its vertex lies in a partition that is not
// resident (it is appended to `out` with that partition).  Moves between
// resident partitions continue in place.
template <uint32_t ALGO, uint32_t SMP>
__global__ void __launch_bounds__(256) k_disk_walk(SlotsDev S, WalkDev a, const uint16_t *__restrict__ vslot,
                                                   const DRec *__restrict__ in, uint32_t n_in,
                                                   const int32_t *__restrict__ vstart, uint32_t parts,
                                                   DRec *__restrict__ out, uint32_t *count_out) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = 0; base < n_in; base += stride) {
        const uint32_t idx = base + blockIdx.x * blockDim.x + threadIdx.x;
        bool leave = false;
        DRec rc{0u, 0, 0u, 0u, -1, {0u, 0u, 0u}};
        if (idx < n_in) {
            rc = in[idx];
            const uint64_t qid = a.qid_base + rc.qi;
            int32_t *__restrict__ path = a.paths + (uint64_t)rc.qi * a.stride;
            uint8_t st = 0;
            for (;;) {
                const uint16_t slot = vslot[rc.cur];
                if (slot == kNoSlot) {
                    leave = true;
                    break;
                }
                GraphDev g;
                TableDev t{};
                slot_views(S, slot, g, t, SMP);
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

// Node2Vec O-REJ move with cur's row in one slot and prev's row in another:
// the darts over cur's row, and for a dart whose height lies between the two
// thresholds it could be judged by, the adjacency test by binary search in
// prev's sorted row.  The darts, thresholds and acceptance are those of the
// in-memory walk without an index (the Node2Vec transition equation; the
// first move takes its first dart).
__device__ __forceinline__ int32_t disk_n2v_move(const int32_t *__restrict__ colc, int32_t off, uint32_t d,
                                                 const int32_t *__restrict__ colp, int32_t poff, int32_t pd,
                                                 const WalkDev &a, uint64_t qid, uint32_t k, int32_t prev,
                                                 const Rand4 &r) {
    Rand4 rr = r;
    for (uint32_t dart = 0;; ++dart) {
        if (dart > 0) rr = philox(k, dart, qid, a.seed);
        const int32_t x = colc[(uint32_t)off + scale32(rr.r0, d)];
        bool accept = (k == 0 || dart + 1 == kMaxDarts);
        if (!accept) {
            const uint32_t y = rr.r1 >> 16;
            if (x == prev) accept = y < a.thr[0];
            else if (y < min(a.thr[1], a.thr[2])) accept = true;
            else if (y >= max(a.thr[1], a.thr[2])) accept = false;
            else accept = y < (in_row(colp, poff, poff + pd, x) ? a.thr[1] : a.thr[2]);
        }
        if (accept) return x;
    }
}

// Node2Vec walkers of one resident pair: each moves while its current and
// previous vertices' partitions are both resident, then ends or waits under
// its new pair.
__global__ void __launch_bounds__(256) k_disk_walk_n2v(SlotsDev S, WalkDev a, const uint16_t *__restrict__ vslot,
                                                       const DRec *__restrict__ in, uint32_t n_in,
                                                       const int32_t *__restrict__ vstart, uint32_t parts,
                                                       DRec *__restrict__ out, uint32_t *count_out) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = 0; base < n_in; base += stride) {
        const uint32_t idx = base + blockIdx.x * blockDim.x + threadIdx.x;
        bool leave = false;
        DRec rc{0u, 0, 0u, 0u, -1, {0u, 0u, 0u}};
        if (idx < n_in) {
            rc = in[idx];
            const uint64_t qid = a.qid_base + rc.qi;
            int32_t *__restrict__ path = a.paths + (uint64_t)rc.qi * a.stride;
            uint8_t st = 0;
            for (;;) {
                const uint16_t sc = vslot[rc.cur];
                const uint16_t sp = rc.prev >= 0 ? vslot[rc.prev] : sc;
                if (sc == kNoSlot || sp == kNoSlot) {
                    leave = true;
                    break;
                }
                const char *bc = S.base + (uint64_t)sc * S.stride;
                const int32_t *rpc = reinterpret_cast<const int32_t *>(bc + S.o_rp);
                const int32_t *colc = reinterpret_cast<const int32_t *>(bc + S.o_col);
                const int32_t off = rpc[rc.cur];
                const uint32_t d = (uint32_t)(rpc[rc.cur + 1] - off);
                int32_t nxt = -1;
                if (d != 0) {
                    const Rand4 r = philox(rc.k, 0, qid, a.seed);
                    const int32_t *colp = colc;
                    int32_t poff = 0, pd = 0;
                    if (rc.prev >= 0) {
                        const char *bp = S.base + (uint64_t)sp * S.stride;
                        const int32_t *rpp = reinterpret_cast<const int32_t *>(bp + S.o_rp);
                        colp = reinterpret_cast<const int32_t *>(bp + S.o_col);
                        poff = rpp[rc.prev];
                        pd = rpp[rc.prev + 1] - poff;
                    }
                    nxt = disk_n2v_move(colc, off, d, colp, poff, pd, a, qid, rc.k, rc.prev, r);
                }
                if (nxt < 0) {
                    st = ST_DEAD_END;
                    break;
                }
                path[rc.k + 1] = nxt;
                ++rc.k;
                if (rc.k == a.max_len) {
                    st = ST_LENGTH;
                    break;
                }
                rc.prev = rc.cur;
                rc.cur = nxt;
            }
            if (leave) {
                const uint32_t pc = part_of(vstart, parts, rc.cur);
                rc.part = pc * parts + (rc.prev >= 0 ? part_of(vstart, parts, rc.prev) : pc);
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

// Table parts for partitions of up to mp edges: total, and the offsets of
// the second and third parts (REJ: p*; ITS: next-slot records, W).
size_t table_bytes(uint32_t algo, uint32_t sampler, int64_t mp, int64_t n, size_t *o1, size_t *o2) {
    *o1 = *o2 = 0;
    if (algo == TRW_A_METAPATH) return 0;
    switch (sampler) {
        case TRW_S_ALIAS: return kAliasEntryBytes * (size_t)mp;
        case TRW_S_ITS:
            *o1 = its_prefix_bytes(mp);
            *o2 = *o1 + its_next_bytes(mp);
            return *o2 + sizeof(uint64_t) * (size_t)n;
        case TRW_S_REJ:
            *o1 = rej_records_bytes(mp);
            return *o1 + sizeof(uint32_t) * (size_t)n;
        default: return 0;
    }
}

// Resident partitions: slots within 1 .. parts; Node2Vec needs two (its
// current and previous vertices' partitions) when there are two.
uint32_t clamp_slots(const trw_disk_graph_s &g, const trw_walk_params &p, uint32_t slots) {
    const uint32_t parts = (uint32_t)(g.vstart.size() - 1);
    const uint32_t least = p.algo == TRW_A_NODE2VEC ? 2u : 1u;
    return std::min<uint32_t>(std::max<uint32_t>(least, std::min(slots, kMaxSlots)), parts);
}

// Keys the waiting walkers are grouped under: partitions, or for Node2Vec
// pairs of partitions.
uint64_t key_count(const trw_disk_graph_s &g, const trw_walk_params &p) {
    const uint64_t parts = g.vstart.size() - 1;
    return p.algo == TRW_A_NODE2VEC ? parts * parts : parts;
}

// Offsets of the pieces of the device workspace and of the pinned buffer.
struct Layout {
    SlotsDev S;
    size_t slots_bytes, vslot, lists[3], vstart, hist, cursor, new_off, old_off, base, consumed, count, dev_total;
    size_t h_rp, h_col, h_wgt, h_lab, h_hist, h_new_off, h_old_off, h_base, h_consumed, host_total;
};

Layout layout(const trw_disk_graph_s &g, const trw_walk_params &p, uint64_t nq, uint32_t slots) {
    const size_t parts = g.vstart.size() - 1, keys = key_count(g, p);
    const size_t mp = (size_t)g.max_edges;
    const bool w = needs_weights(p.sampler, p.algo), l = p.algo == TRW_A_METAPATH;
    Layout L{};
    size_t o = 0;
    auto take = [&o](size_t bytes) { const size_t at = o; o += r256(bytes); return at; };
    size_t o1 = 0, o2 = 0;
    L.S.o_rp = take(4 * ((size_t)g.n + 1));
    L.S.o_col = take(4 * mp);
    L.S.o_wgt = take(w ? 4 * mp : 0);
    L.S.o_lab = take(l ? mp : 0);
    L.S.o_tab = take(table_bytes(p.algo, p.sampler, (int64_t)mp, g.n, &o1, &o2));
    L.S.stride = o;
    L.S.tab_o1 = o1;
    L.S.tab_o2 = o2;
    L.S.n = (int32_t)g.n;
    L.S.has_wgt = w;
    L.S.has_lab = l;
    L.slots_bytes = o * clamp_slots(g, p, slots);
    o = L.slots_bytes;
    L.vslot = take(2 * (size_t)g.n + 4);
    for (auto &x : L.lists) x = take(sizeof(DRec) * (size_t)nq);
    L.vstart = take(4 * (parts + 1));
    L.hist = take(4 * keys);
    L.cursor = take(4 * keys);
    L.new_off = take(4 * keys);
    L.old_off = take(4 * keys);
    L.base = take(4 * keys);
    L.consumed = take(keys);
    L.count = take(4);
    L.dev_total = o;
    o = 0;
    L.h_rp = take(4 * ((size_t)g.max_verts + 1));
    L.h_col = take(4 * mp);
    L.h_wgt = take(w ? 4 * mp : 0);
    L.h_lab = take(l ? mp : 0);
    L.h_hist = take(4 * keys + 4);
    L.h_new_off = take(4 * keys);
    L.h_old_off = take(4 * keys);
    L.h_base = take(4 * keys);
    L.h_consumed = take(keys);
    L.host_total = o;
    return L;
}

trw_status check_walk(const trw_disk_graph_s *g, const trw_walk_params *p) {
    if (!g) return dfail(TRW_E_INVALID, "disk graph is NULL");
    if (!p) return dfail(TRW_E_INVALID, "params is NULL");
    if (p->algo == TRW_A_NODE2VEC) {
        if (p->sampler != TRW_S_OREJ) return dfail(TRW_E_UNSUPPORTED, "Node2Vec walks with O-REJ");
        for (int i = 0; i < 3; ++i)
            if (p->n2v_thr_q16[i] == 0 || p->n2v_thr_q16[i] > 65536)
                return dfail(TRW_E_INVALID, "Node2Vec thresholds must be in 1..65536");
        if (g->vstart.size() - 1 > kMaxPairParts)
            return dfail(TRW_E_UNSUPPORTED, "Node2Vec from a file takes at most 1024 partitions (its walkers wait "
                                            "under pairs of partitions)");
    } else if (p->algo == TRW_A_DEEPWALK || p->algo == TRW_A_PPR) {
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
void launch_disk_walk(const SlotsDev &S, const WalkDev &w, const uint16_t *vslot, const DRec *in, uint32_t n_in,
                      const int32_t *vstart, uint32_t parts, DRec *out, uint32_t *count, uint32_t blocks,
                      hipStream_t s) {
    hipLaunchKernelGGL((k_disk_walk<ALGO, SMP>), dim3(blocks), dim3(256), 0, s, S, w, vslot, in, n_in, vstart, parts,
                       out, count);
}

void dispatch_walk(uint32_t algo, uint32_t sampler, const SlotsDev &S, const WalkDev &w, const uint16_t *vslot,
                   const DRec *in, uint32_t n_in, const int32_t *vstart, uint32_t parts, DRec *out, uint32_t *count,
                   uint32_t blocks, hipStream_t s) {
#define TRW_DISK_WALK(A, M) launch_disk_walk<A, M>(S, w, vslot, in, n_in, vstart, parts, out, count, blocks, s)
    if (algo == TRW_A_NODE2VEC) {
        hipLaunchKernelGGL(k_disk_walk_n2v, dim3(blocks), dim3(256), 0, s, S, w, vslot, in, n_in, vstart, parts, out,
                           count);
        return;
    }
    if (algo == TRW_A_METAPATH) {
        TRW_DISK_WALK(ALG_METAPATH, SMP_ITS);
        return;
    }
    const bool ppr = algo == TRW_A_PPR;
    switch (sampler) {
        case TRW_S_NAIVE:
            if (ppr) TRW_DISK_WALK(ALG_PPR, SMP_NAIVE); else TRW_DISK_WALK(ALG_DEEPWALK, SMP_NAIVE);
            break;
        case TRW_S_ALIAS:
            if (ppr) TRW_DISK_WALK(ALG_PPR, SMP_ALIAS); else TRW_DISK_WALK(ALG_DEEPWALK, SMP_ALIAS);
            break;
        case TRW_S_REJ:
            if (ppr) TRW_DISK_WALK(ALG_PPR, SMP_REJ); else TRW_DISK_WALK(ALG_DEEPWALK, SMP_REJ);
            break;
        default:
            if (ppr) TRW_DISK_WALK(ALG_PPR, SMP_ITS); else TRW_DISK_WALK(ALG_DEEPWALK, SMP_ITS);
    }
#undef TRW_DISK_WALK
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

static trw_status disk_graph_open(const char *path, uint64_t part_edges, trw_disk_graph *out);

trw_status trw_disk_graph_open(const char *path, uint64_t part_edges, trw_disk_graph *out) {
    try {
        return disk_graph_open(path, part_edges, out);
    } catch (...) {
        return dfail(TRW_E_INVALID, "out of host memory opening the file");
    }
}

static trw_status disk_graph_open(const char *path, uint64_t part_edges, trw_disk_graph *out) {
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
    g->sorted.assign(g->vstart.size() - 1, 0);
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


trw_status trw_disk_walk_bytes(trw_disk_graph g, const trw_walk_params *p, uint64_t nq, uint32_t slots,
                               size_t *device_bytes, size_t *host_bytes) {
    trw_status st = check_walk(g, p);
    if (st != TRW_OK) return st;
    if (!device_bytes || !host_bytes) return dfail(TRW_E_INVALID, "device_bytes / host_bytes is NULL");
    if (nq >= (uint64_t(1) << 32)) return dfail(TRW_E_INVALID, "nq must be < 2^32");
    const Layout L = layout(*g, *p, nq, slots);
    *device_bytes = L.dev_total;
    *host_bytes = L.host_total;
    return TRW_OK;
}

static trw_status disk_walk(trw_disk_graph g, const trw_walk_params *p, const int32_t *d_sources, uint64_t nq,
                            uint64_t qid_base, int32_t *d_paths, uint64_t path_stride, uint32_t *d_lengths,
                            uint8_t *d_status, uint32_t slots, void *d_ws, size_t ws_bytes, void *h_pinned,
                            size_t h_bytes, trw_disk_walk_stats *stats, trw_stream_t stream);

trw_status trw_disk_walk(trw_disk_graph g, const trw_walk_params *p, const int32_t *d_sources, uint64_t nq,
                         uint64_t qid_base, int32_t *d_paths, uint64_t path_stride, uint32_t *d_lengths,
                         uint8_t *d_status, uint32_t slots, void *d_ws, size_t ws_bytes, void *h_pinned,
                         size_t h_bytes, trw_disk_walk_stats *stats, trw_stream_t stream) {
    try {
        return disk_walk(g, p, d_sources, nq, qid_base, d_paths, path_stride, d_lengths, d_status, slots, d_ws,
                         ws_bytes, h_pinned, h_bytes, stats, stream);
    } catch (...) {
        (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
        return dfail(TRW_E_INVALID, "out of host memory during the walk");
    }
}

static trw_status disk_walk(trw_disk_graph g, const trw_walk_params *p, const int32_t *d_sources, uint64_t nq,
                            uint64_t qid_base, int32_t *d_paths, uint64_t path_stride, uint32_t *d_lengths,
                            uint8_t *d_status, uint32_t slots, void *d_ws, size_t ws_bytes, void *h_pinned,
                            size_t h_bytes, trw_disk_walk_stats *stats, trw_stream_t stream) {
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
    const uint32_t K = clamp_slots(*g, *p, slots);
    const bool pairs = p->algo == TRW_A_NODE2VEC;
    const uint32_t keys = (uint32_t)key_count(*g, *p);
    Layout L = layout(*g, *p, nq, K);
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
    const size_t lds_hist = keys <= kLdsParts ? 4 * (size_t)keys : 0;   // the regroup kernels' LDS counts
    L.S.base = D;
    const SlotsDev &SD = L.S;

    uint16_t *d_vslot = reinterpret_cast<uint16_t *>(D + L.vslot);
    DRec *lists[3] = {reinterpret_cast<DRec *>(D + L.lists[0]), reinterpret_cast<DRec *>(D + L.lists[1]),
                      reinterpret_cast<DRec *>(D + L.lists[2])};
    int32_t *d_vstart = reinterpret_cast<int32_t *>(D + L.vstart);
    uint32_t *d_hist = reinterpret_cast<uint32_t *>(D + L.hist);
    uint32_t *d_cursor = reinterpret_cast<uint32_t *>(D + L.cursor);
    uint32_t *d_new_off = reinterpret_cast<uint32_t *>(D + L.new_off);
    uint32_t *d_old_off = reinterpret_cast<uint32_t *>(D + L.old_off);
    uint32_t *d_base = reinterpret_cast<uint32_t *>(D + L.base);
    uint8_t *d_consumed = reinterpret_cast<uint8_t *>(D + L.consumed);
    uint32_t *d_count = reinterpret_cast<uint32_t *>(D + L.count);
    int32_t *h_rp = reinterpret_cast<int32_t *>(H + L.h_rp);
    char *h_col = H + L.h_col;
    char *h_wgt = H + L.h_wgt;
    char *h_lab = H + L.h_lab;
    uint32_t *h_hist = reinterpret_cast<uint32_t *>(H + L.h_hist);   // key counts, then the arrival count
    uint32_t *h_new_off = reinterpret_cast<uint32_t *>(H + L.h_new_off);
    uint32_t *h_old_off = reinterpret_cast<uint32_t *>(H + L.h_old_off);
    uint32_t *h_base = reinterpret_cast<uint32_t *>(H + L.h_base);
    uint8_t *h_consumed = reinterpret_cast<uint8_t *>(H + L.h_consumed);

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
    auto set_slot = [&](int64_t lo, int64_t hi, uint16_t v) {
        if (hi > lo)
            hipLaunchKernelGGL(k_disk_set_slot, dim3(grid_for((uint64_t)(hi - lo), di)), dim3(256), 0, s, d_vslot, lo,
                               hi, v);
    };
    // histogram of the arrivals in lists[2] (count in d_count) into h_hist; waits
    auto read_arrivals = [&]() {
        fill(d_hist, keys, 0u);
        hipLaunchKernelGGL(k_disk_hist, dim3(grid_for(nq, di)), dim3(256), lds_hist, s, lists[2], d_count, d_hist,
                           keys);
        e = hipMemcpyAsync(h_hist, d_hist, 4 * (size_t)keys, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h_hist + keys, d_count, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e == hipSuccess;
    };
    // file bytes [foff, foff + bytes) to device memory through the pinned
    // staging area, in chunks: each chunk's copy runs while the next is read
    auto stream_in = [&](char *hbuf, char *dbuf, size_t bytes, uint64_t foff, bool check_cols, int64_t e0) -> bool {
        for (size_t o = 0; o < bytes; o += kReadChunk) {
            const size_t b = std::min(kReadChunk, bytes - o);
            const uint64_t t0 = now_ns();
            const bool ok = read_parallel(g->fd, hbuf + o, b, foff + o);
            S.read_ns += now_ns() - t0;
            if (!ok) {
                set_error("cannot read the file");
                return false;
            }
            S.bytes_read += b;
            if (check_cols) {
                const int32_t *c = reinterpret_cast<const int32_t *>(hbuf + o);
                for (size_t i = 0; i < b / 4; ++i)
                    if ((uint32_t)c[i] >= (uint32_t)g->n) {
                        set_error("edge " + std::to_string(e0 + (int64_t)(o / 4 + i)) +
                                  " has a destination outside [0, n)");
                        return false;
                    }
            }
            e = hipMemcpyAsync(dbuf + o, hbuf + o, b, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) {
                set_error(std::string("partition copy: ") + hipGetErrorString(e));
                return false;
            }
        }
        return true;
    };

    // partition starts on the device (int32: n < 2^31); no vertex resident
    {
        std::vector<int32_t> vs(g->vstart.begin(), g->vstart.end());
        e = hipMemcpyAsync(d_vstart, vs.data(), 4 * vs.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return device_error("partition starts upload");
    }
    set_slot(0, g->n, kNoSlot);
    // the sources wait in their partitions
    fill(d_count, 1, 0u);
    hipLaunchKernelGGL(k_disk_init, dim3(grid_for(nq, di)), dim3(256), 0, s, w, (int32_t)g->n, d_vstart, parts,
                       (uint32_t)pairs, lists[2], d_count);
    e = hipGetLastError();
    if (e != hipSuccess || !read_arrivals()) return device_error("start");

    // host copies of the waiting list's layout: per key its count and start
    std::vector<uint64_t> counts(keys, 0), next(keys, 0), off(keys, 0);
    std::vector<uint8_t> consumed(keys, 0);
    // resident partitions: slot -> partition, partition -> slot, last round used
    std::vector<int64_t> slot_part(K, -1), slot_used(K, -1);
    std::vector<int32_t> part_slot(parts, -1);
    DRec *cur = lists[0], *spare = lists[1];
    uint64_t old_total = 0, round = 0, moved_max = nq * (uint64_t)p->max_len;

    // Load partition q into the slot used longest ago that does not hold
    // `keep` (the other partition a Node2Vec pair needs): its rows, its edges
    // (checked on the first load), its table.
    auto load = [&](uint32_t q, uint32_t keep) -> trw_status {
        // the pinned staging area is refilled below: the copies of a load just
        // made (a Node2Vec pair loads two partitions in one round) must be done
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return device_error("partition copy");
        uint32_t slot = K;
        for (uint32_t k = 0; k < K; ++k)
            if (slot_part[k] != (int64_t)keep && (slot == K || slot_used[k] < slot_used[slot])) slot = k;
        const int64_t v0 = g->vstart[q], v1 = g->vstart[q + 1];
        const int64_t e0 = g->row_ptr[v0], e1 = g->row_ptr[v1];
        const int64_t mp = e1 - e0;
        if (slot_part[slot] >= 0) {
            const int64_t old = slot_part[slot];
            set_slot(g->vstart[old], g->vstart[old + 1], kNoSlot);
            part_slot[old] = -1;
            slot_part[slot] = -1;
        }
        char *b = D + (uint64_t)slot * SD.stride;
        int32_t *d_rp = reinterpret_cast<int32_t *>(b + SD.o_rp);
        char *d_tab = b + SD.o_tab;
        for (int64_t v = v0; v <= v1; ++v) h_rp[v - v0] = (int32_t)(g->row_ptr[v] - e0);
        hipLaunchKernelGGL(k_disk_rows, dim3(grid_for((uint64_t)g->n + 1, di)), dim3(256), 0, s, d_rp, g->n, v0, v1,
                           (int32_t)mp);
        e = hipMemcpyAsync(d_rp + v0, h_rp, 4 * (size_t)(v1 - v0 + 1), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return device_error("partition copy");
        bool ok = stream_in(h_col, b + SD.o_col, 4 * (size_t)mp, g->off_col + 4 * (uint64_t)e0, !g->checked[q], e0);
        if (ok && want_w)
            ok = stream_in(h_wgt, b + SD.o_wgt, 4 * (size_t)mp, g->off_weight + 4 * (uint64_t)e0, false, e0);
        if (ok && want_l) ok = stream_in(h_lab, b + SD.o_lab, (size_t)mp, g->off_label + (uint64_t)e0, false, e0);
        if (!ok) {
            if (e != hipSuccess) return device_error("partition copy");
            (void)hipStreamSynchronize(s);
            return TRW_E_INVALID;   // the message is set
        }
        g->checked[q] = 1;
        if (pairs && g->sorted[q] == 0) {
            // the adjacency test searches rows: each must be sorted
            const int32_t *c = reinterpret_cast<const int32_t *>(h_col);
            g->sorted[q] = 1;
            for (int64_t v = v0; v < v1 && g->sorted[q] == 1; ++v)
                for (int64_t x = g->row_ptr[v] - e0 + 1; x < g->row_ptr[v + 1] - e0; ++x)
                    if (c[x - 1] > c[x]) {
                        g->sorted[q] = 2;
                        break;
                    }
        }
        if (pairs && g->sorted[q] == 2)
            return host_error("Node2Vec searches rows: a row of partition " + std::to_string(q) + " is not sorted");
        if (mp > 0 && p->algo != TRW_A_METAPATH && p->algo != TRW_A_NODE2VEC) {
            GraphDev view{d_rp, reinterpret_cast<const int32_t *>(b + SD.o_col),
                          want_w ? reinterpret_cast<const uint32_t *>(b + SD.o_wgt) : nullptr, nullptr,
                          (int32_t)g->n, (int32_t)mp, 0};
            if (p->sampler == TRW_S_ALIAS)
                e = launch_alias_build_range(view, v0, v1, reinterpret_cast<uint4 *>(d_tab), s);
            else if (p->sampler == TRW_S_ITS)
                e = launch_its_build_range(view, v0, v1, reinterpret_cast<uint64_t *>(d_tab),
                                           reinterpret_cast<uint4 *>(d_tab + SD.tab_o1),
                                           reinterpret_cast<uint64_t *>(d_tab + SD.tab_o2), s);
            else if (p->sampler == TRW_S_REJ)
                e = launch_rej_build_range(view, v0, v1, reinterpret_cast<uint4 *>(d_tab),
                                           reinterpret_cast<uint32_t *>(d_tab + SD.tab_o1), s);
            if (e != hipSuccess) return device_error("table build launch");
        }
        set_slot(v0, v1, (uint16_t)slot);
        slot_part[slot] = q;
        part_slot[q] = (int32_t)slot;
        slot_used[slot] = (int64_t)round;
        ++S.loads;
        return TRW_OK;
    };

    for (;;) {
        // regroup into `spare`: each key's old records (none for those just
        // walked), then its arrivals.  The pinned arrays are written here
        // only, after the previous round's wait, and read by this round's copies.
        uint64_t acc = 0, old_kept = 0;
        for (uint32_t q = 0; q < keys; ++q) {
            const uint64_t kept = consumed[q] ? 0 : counts[q];
            old_kept += kept;
            next[q] = kept + h_hist[q];
            h_old_off[q] = (uint32_t)off[q];
            h_new_off[q] = (uint32_t)acc;
            h_base[q] = (uint32_t)(acc + kept);
            h_consumed[q] = consumed[q];
            acc += next[q];
        }
        const uint64_t waiting = acc;
        e = hipMemcpyAsync(d_new_off, h_new_off, 4 * (size_t)keys, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_base, h_base, 4 * (size_t)keys, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && old_kept > 0)
            e = hipMemcpyAsync(d_old_off, h_old_off, 4 * (size_t)keys, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && old_kept > 0) e = hipMemcpyAsync(d_consumed, h_consumed, keys, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return device_error("offsets upload");
        if (old_kept > 0)
            hipLaunchKernelGGL(k_disk_move_old, dim3(grid_for(old_total, di)), dim3(256), 0, s, cur,
                               (uint32_t)old_total, d_consumed, d_old_off, d_new_off, spare);
        fill(d_cursor, keys, 0u);
        hipLaunchKernelGGL(k_disk_place_new, dim3(grid_for(h_hist[keys], di)), dim3(256), 2 * lds_hist, s, lists[2],
                           d_count, d_base, d_cursor, spare, keys);
        e = hipGetLastError();
        if (e != hipSuccess) return device_error("regroup launch");
        std::swap(cur, spare);
        counts.swap(next);
        for (uint32_t q = 0; q < keys; ++q) off[q] = h_new_off[q];
        old_total = waiting;
        if (waiting == 0) break;
        // Each round moves every walker it runs at least once or ends it, so
        // there are at most nq * max_len rounds.
        if (++round > moved_max) return host_error("partition walks made no progress");

        // run the keys whose partitions are resident; if none holds a waiting
        // query, load the partitions of the key holding the most (the lowest
        // index among equals)
        std::vector<uint32_t> resident, run;
        for (uint32_t k = 0; k < K; ++k)
            if (slot_part[k] >= 0) resident.push_back((uint32_t)slot_part[k]);
        for (uint32_t a : resident) {
            if (!pairs) {
                if (counts[a] > 0) run.push_back(a);
                continue;
            }
            for (uint32_t b : resident)
                if (counts[(uint64_t)a * parts + b] > 0) run.push_back(a * parts + b);
        }
        if (run.empty()) {
            uint32_t best = 0;
            for (uint32_t q = 1; q < keys; ++q)
                if (counts[q] > counts[best]) best = q;
            const uint32_t a = pairs ? best / parts : best, b = pairs ? best % parts : best;
            if (part_slot[a] < 0 && (st = load(a, b)) != TRW_OK) return st;
            if (part_slot[b] < 0 && (st = load(b, a)) != TRW_OK) return st;
            run.push_back(best);
        }
        // walk every query waiting under them; those that step out of the
        // resident partitions arrive in lists[2]
        ++S.runs;
        fill(d_count, 1, 0u);
        std::fill(consumed.begin(), consumed.end(), 0);
        for (uint32_t q : run) {
            const uint32_t n_in = (uint32_t)counts[q];
            dispatch_walk(p->algo, p->sampler, SD, w, d_vslot, cur + off[q], n_in, d_vstart, parts, lists[2], d_count,
                          grid_for(n_in, di), s);
            consumed[q] = 1;
            slot_used[part_slot[pairs ? q / parts : q]] = (int64_t)round;
            slot_used[part_slot[pairs ? q % parts : q]] = (int64_t)round;
        }
        e = hipGetLastError();
        if (e != hipSuccess || !read_arrivals()) return device_error("partition walk");
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error("finish");
    S.total_ns = now_ns() - t_start;
    if (stats) *stats = S;
    return TRW_OK;
}

}  // extern "C"
