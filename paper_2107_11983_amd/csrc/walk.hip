// The Gather-Move-Update walk step on CDNA4 (gfx950).
//
// One walker per lane.  Each step of a walker (Step-centric Programming, the
// framework algorithm) reads the current vertex's row range (Gather; for
// static walks the per-vertex table built beforehand replaces the gather),
// draws one Philox block keyed by (seed, query, move), samples the next vertex
// (Move) and appends it, then applies the termination rule (Update).
//
// Two schedules:
//  * persistent: one launch.  Each wave claims chunks of query ids from a
//    device queue; a lane whose walk ends takes the next id from its wave's
//    chunk (ballot + mbcnt rank), so lanes stay busy however uneven the walk
//    lengths are.  GPU occupancy plays the part of the paper's step
//    interleaving: many independent walkers per CU keep many random reads in
//    flight.  Optionally each lane interleaves 2 or 4 walkers.
//  * per step (bulk-synchronous): one launch per move over a compacted list
//    of live walker records; finished walkers drop out of the next list.
//
// Memory traffic per move is what bounds the step (random reads fetch whole
// cache lines).  ALIAS entries carry the row range of both candidate
// destinations, so an ALIAS move is a single random 32-byte read; path
// entries are buffered in registers and written 16 bytes at a time on 16-byte
// boundaries of the path row.
//
// Sampling is integer throughout: uniform index = high half of r * d; ALIAS
// coin r1 < thr; ITS draw = high half of (r1:r0) * W and a binary search over
// the uint64 prefix; O-REJ darts compare r1 >> 16 with Q16 thresholds;
// MetaPath counts the matching labels of the row and takes the j-th.
#include "trw_device.hpp"
#include "trw_internal.hpp"

namespace trw {
namespace {

constexpr uint32_t kIdle = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Move for the samplers that read the adjacency array (NAIVE, ITS, O-REJ,
// MetaPath).  Returns the next vertex, or -1 when the current vertex has no
// eligible edge (dead end).  `r` is the block of dart 0.
// ---------------------------------------------------------------------------
template <uint32_t ALGO, uint32_t SMP>
__device__ __forceinline__ int32_t sample_next(const GraphDev &g, const TableDev &t, const WalkDev &a,
                                               uint64_t qid, uint32_t k, int32_t off, uint32_t d,
                                               const Rand4 &r, int32_t prev, int32_t poff, int32_t pd) {
    if (ALGO == ALG_NODE2VEC) {
        // O-REJ with p* = max weight: throw darts (x, y) until y < p(x) / p*.
        Rand4 rr = r;
        for (uint32_t dart = 0;; ++dart) {
            if (dart > 0) rr = philox(k, dart, qid, a.seed);
            const int32_t x = g.col[off + scale32(rr.r0, d)];
            if (k == 0 || dart + 1 == kMaxDarts) return x;
            uint32_t th;
            if (x == prev) {
                th = a.thr[0];
            } else {
                // is x adjacent to prev?  binary search in prev's sorted row
                int32_t lo = poff, hi = poff + pd;
                bool found = false;
                while (lo < hi) {
                    const int32_t mid = lo + ((hi - lo) >> 1);
                    const int32_t c = g.col[mid];
                    if (c == x) { found = true; break; }
                    if (c < x) lo = mid + 1; else hi = mid;
                }
                th = found ? a.thr[1] : a.thr[2];
            }
            if ((rr.r1 >> 16) < th) return x;
        }
    } else if (ALGO == ALG_METAPATH) {
        const uint32_t si = k % a.schema_len;
        const uint64_t word = si < 8 ? a.schema_lo : a.schema_hi;
        const uint8_t want = (uint8_t)(word >> ((si & 7u) * 8u));
        const uint8_t *__restrict__ lab = g.label + off;
        uint32_t m = 0;
        for (uint32_t i = 0; i < d; ++i) m += (lab[i] == want);
        if (m == 0) return -1;
        uint32_t j = scale32(r.r0, m);
        for (uint32_t i = 0;; ++i) {
            if (lab[i] == want) {
                if (j == 0) return g.col[off + i];
                --j;
            }
        }
    } else if (SMP == SMP_NAIVE) {
        return g.col[off + scale32(r.r0, d)];
    } else {  // ITS
        const uint64_t *__restrict__ p = t.prefix + off;
        const uint64_t W = p[d - 1];
        if (W == 0) return -1;
        const uint64_t x = scale64(r.r0, r.r1, W);
        uint32_t lo = 0, hi = d - 1;                          // smallest i with x < p[i]
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (x < p[mid]) hi = mid; else lo = mid + 1;
        }
        return g.col[off + lo];
    }
}

// ALIAS move from the 32-byte entry of column j: next vertex and its row range.
__device__ __forceinline__ int32_t alias_pick(const uint4 &e0, const uint4 &e1, uint32_t r1, int32_t &off,
                                              int32_t &deg) {
    const bool first = r1 < e0.x;
    off = (int32_t)(first ? e1.x : e1.z);
    deg = (int32_t)(first ? e1.y : e1.w);
    return (int32_t)(first ? e0.y : e0.z);                  // -1 marks a row of zero weight
}

// ---------------------------------------------------------------------------
// Path writer: up to 4 pending entries per walker, flushed as one 16-byte
// store when they end on a 16-byte boundary, else entry by entry at the end.
// ---------------------------------------------------------------------------
struct PathBuf {
    int32_t *p;      // address of the first pending entry
    uint32_t n;      // pending entries
    int32_t b0, b1, b2, b3;

    __device__ __forceinline__ void start(int32_t *row) { p = row; n = 0; }

    __device__ __forceinline__ void flush() {
        if (n == 4) {
            *reinterpret_cast<int4 *>(p) = make_int4(b0, b1, b2, b3);
        } else {
            if (n > 0) p[0] = b0;
            if (n > 1) p[1] = b1;
            if (n > 2) p[2] = b2;
        }
        p += n;
        n = 0;
    }

    __device__ __forceinline__ void push(int32_t v) {
        if (n == 0) b0 = v; else if (n == 1) b1 = v; else if (n == 2) b2 = v; else b3 = v;
        ++n;
        if (((reinterpret_cast<uintptr_t>(p + n)) & 15u) == 0) flush();
    }
};

// ---------------------------------------------------------------------------
// Persistent schedule
// ---------------------------------------------------------------------------
struct Walker {
    uint32_t qi;     // index in the batch, kIdle when the slot is free
    int32_t cur;
    int32_t prev;
    uint32_t k;
    int32_t off;     // row of cur (valid when !need_row)
    int32_t deg;
    int32_t poff;    // row of prev (Node2Vec)
    int32_t pdeg;
    bool need_row;
    PathBuf path;
};

template <uint32_t ALGO, uint32_t SMP, int WPL>
__global__ void __launch_bounds__(256)
k_walk_persistent(GraphDev g, TableDev t, WalkDev a, unsigned long long *__restrict__ queue_head,
                  uint32_t chunk) {
    constexpr bool kAlias = (SMP == SMP_ALIAS) && (ALGO == ALG_DEEPWALK || ALGO == ALG_PPR);
    Walker w[WPL];
#pragma unroll
    for (int i = 0; i < WPL; ++i) w[i].qi = kIdle;
    uint32_t pool_next = 0, pool_end = 0;   // this wave's claimed id range (wave-uniform)
    bool exhausted = false;
    const uint32_t lane = lane_id();
    const unsigned long long n_waves = ((unsigned long long)gridDim.x * blockDim.x + 63) / 64;
    unsigned long long seen = 0;            // queue head after this wave's last claim (wave-uniform)

    for (;;) {
        // Admission / refill: idle slots take the next ids of the wave's chunk.
        for (int i = 0; i < WPL; ++i) {
            uint64_t idle = __ballot(w[i].qi == kIdle);
            while (idle != 0 && !exhausted) {
                uint32_t avail = pool_end - pool_next;
                if (avail == 0) {
                    // Guided claim: a share of what was left at this wave's previous claim,
                    // between 64 ids and `chunk`, so that early claims are large (few
                    // atomics) and late ones small (waves finish together).
                    const unsigned long long left = seen < a.nq ? a.nq - seen : 0;
                    uint32_t take = (uint32_t)min(left / (2ull * n_waves), (unsigned long long)chunk);
                    take = max(take, min(64u, chunk));
                    unsigned long long base = 0;
                    if (lane == 0) base = atomicAdd(queue_head, (unsigned long long)take);
                    base = __shfl(base, 0);
                    seen = base + take;
                    if (base >= a.nq) { exhausted = true; break; }
                    pool_next = (uint32_t)base;
                    pool_end = (uint32_t)min(base + take, (unsigned long long)a.nq);
                    avail = pool_end - pool_next;
                }
                const uint32_t rk = rank_below(idle);
                if (((idle >> lane) & 1ull) && rk < avail) {
                    const uint32_t qi = pool_next + rk;
                    const int32_t s = a.sources[qi];
                    if (s < 0 || s >= g.n) {
                        a.lengths[qi] = 0;
                        a.status[qi] = ST_BAD_SOURCE;
                    } else {
                        w[i].qi = qi; w[i].cur = s; w[i].prev = -1; w[i].k = 0;
                        w[i].poff = 0; w[i].pdeg = 0; w[i].need_row = true;
                        w[i].path.start(a.paths + (uint64_t)qi * a.stride);
                        w[i].path.push(s);
                    }
                }
                pool_next += min((uint32_t)__popcll(idle), avail);
                idle = __ballot(w[i].qi == kIdle);
            }
        }
        bool any = false;
#pragma unroll
        for (int i = 0; i < WPL; ++i) any |= (w[i].qi != kIdle);
        if (__ballot(any) == 0) break;   // every slot idle after refill: the queue is drained

        // Gather: row ranges the walkers do not carry yet (independent loads).
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            if (w[i].qi != kIdle && w[i].need_row) {
                const int32_t lo = g.row_ptr[w[i].cur];
                w[i].deg = g.row_ptr[w[i].cur + 1] - lo;
                w[i].off = lo;
                w[i].need_row = false;
            }
        }
        Rand4 r[WPL];
#pragma unroll
        for (int i = 0; i < WPL; ++i) r[i] = philox(w[i].k, 0, a.qid_base + w[i].qi, a.seed);

        // Move.
        int32_t nxt[WPL];
        if (kAlias) {
            uint4 e0[WPL], e1[WPL];
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                if (w[i].qi != kIdle && w[i].deg != 0) {
                    const uint32_t e = (uint32_t)w[i].off + scale32(r[i].r0, (uint32_t)w[i].deg);
                    e0[i] = t.alias[2 * (uint64_t)e];
                    e1[i] = t.alias[2 * (uint64_t)e + 1];
                }
            }
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                nxt[i] = -1;
                if (w[i].qi != kIdle && w[i].deg != 0) {
                    w[i].poff = w[i].off; w[i].pdeg = w[i].deg;
                    nxt[i] = alias_pick(e0[i], e1[i], r[i].r1, w[i].off, w[i].deg);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                nxt[i] = -1;
                if (w[i].qi != kIdle && w[i].deg != 0) {
                    nxt[i] = sample_next<ALGO, SMP>(g, t, a, a.qid_base + w[i].qi, w[i].k, w[i].off,
                                                    (uint32_t)w[i].deg, r[i], w[i].prev, w[i].poff, w[i].pdeg);
                    w[i].poff = w[i].off; w[i].pdeg = w[i].deg;
                    w[i].need_row = true;
                }
            }
        }

        // Update.
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            if (w[i].qi == kIdle) continue;
            uint8_t st = 0;
            if (nxt[i] < 0) {
                st = ST_DEAD_END;
            } else {
                w[i].path.push(nxt[i]);
                w[i].prev = w[i].cur;
                w[i].cur = nxt[i];
                w[i].k += 1;
                if (ALGO == ALG_PPR && r[i].r2 < a.stop_q32) st = ST_STOPPED;
                else if (w[i].k == a.max_len) st = ST_LENGTH;
            }
            if (st) {
                w[i].path.flush();
                a.lengths[w[i].qi] = w[i].k;
                a.status[w[i].qi] = st;
                w[i].qi = kIdle;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Per-step (bulk-synchronous) schedule
// ---------------------------------------------------------------------------
// A live walker between launches: query index, current vertex and two words
// that are the row range of cur for ALIAS walks, and (prev, unused) otherwise.
struct alignas(16) Rec {
    uint32_t qi;
    int32_t cur;
    int32_t a;
    int32_t b;
};

__global__ void k_fill_u32(uint32_t *p, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <bool ALIAS_ROWS>
__global__ void __launch_bounds__(256) k_bsp_init(GraphDev g, WalkDev a, Rec *__restrict__ out,
                                                  uint32_t *__restrict__ count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = 0; base < a.nq; base += stride) {
        const uint64_t i = base + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        bool keep = false;
        int32_t s = 0;
        if (i < a.nq) {
            s = a.sources[i];
            if (s < 0 || s >= g.n) {
                a.lengths[i] = 0;
                a.status[i] = ST_BAD_SOURCE;
            } else {
                a.paths[i * a.stride] = s;
                keep = true;
            }
        }
        const uint32_t slot = wave_append(count, keep);
        if (keep) {
            if (ALIAS_ROWS) {
                const int32_t lo = g.row_ptr[s];
                out[slot] = Rec{(uint32_t)i, s, lo, g.row_ptr[s + 1] - lo};
            } else {
                out[slot] = Rec{(uint32_t)i, s, -1, 0};
            }
        }
    }
}

template <uint32_t ALGO, uint32_t SMP>
__global__ void __launch_bounds__(256) k_bsp_step(GraphDev g, TableDev t, WalkDev a, uint32_t k,
                                                  const Rec *__restrict__ in, const uint32_t *__restrict__ count_in,
                                                  Rec *__restrict__ out, uint32_t *__restrict__ count_out) {
    constexpr bool kAlias = (SMP == SMP_ALIAS) && (ALGO == ALG_DEEPWALK || ALGO == ALG_PPR);
    const uint32_t n_in = *count_in;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = 0; base < n_in; base += stride) {
        const uint32_t idx = base + blockIdx.x * blockDim.x + threadIdx.x;
        bool keep = false;
        Rec nr{};
        if (idx < n_in) {
            const Rec rc = in[idx];
            const uint64_t qid = a.qid_base + rc.qi;
            const Rand4 r = philox(k, 0, qid, a.seed);
            int32_t nxt = -1, noff = 0, ndeg = 0;
            if (kAlias) {
                if (rc.b != 0) {
                    const uint32_t e = (uint32_t)rc.a + scale32(r.r0, (uint32_t)rc.b);
                    nxt = alias_pick(t.alias[2 * (uint64_t)e], t.alias[2 * (uint64_t)e + 1], r.r1, noff, ndeg);
                }
            } else {
                const int32_t off = g.row_ptr[rc.cur];
                const uint32_t d = (uint32_t)(g.row_ptr[rc.cur + 1] - off);
                int32_t poff = 0, pd = 0;
                if (ALGO == ALG_NODE2VEC && rc.a >= 0) {
                    poff = g.row_ptr[rc.a];
                    pd = g.row_ptr[rc.a + 1] - poff;
                }
                if (d != 0) nxt = sample_next<ALGO, SMP>(g, t, a, qid, k, off, d, r, rc.a, poff, pd);
            }
            uint8_t st = 0;
            uint32_t len = k;
            if (nxt < 0) {
                st = ST_DEAD_END;
            } else {
                a.paths[(uint64_t)rc.qi * a.stride + k + 1] = nxt;
                len = k + 1;
                if (ALGO == ALG_PPR && r.r2 < a.stop_q32) st = ST_STOPPED;
                else if (len == a.max_len) st = ST_LENGTH;
            }
            if (st) {
                a.lengths[rc.qi] = len;
                a.status[rc.qi] = st;
            } else {
                keep = true;
                nr = kAlias ? Rec{rc.qi, nxt, noff, ndeg} : Rec{rc.qi, nxt, rc.cur, 0};
            }
        }
        const uint32_t slot = wave_append(count_out, keep);
        if (keep) out[slot] = nr;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
constexpr size_t kAlign = 256;
inline size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

template <uint32_t ALGO, uint32_t SMP>
hipError_t run_persistent(const GraphDev &g, const TableDev &t, const WalkDev &w, const Tuning &tu,
                          const DeviceInfo &di, void *ws, hipStream_t s) {
    auto *head = reinterpret_cast<unsigned long long *>(ws);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(ws), 2u, 0u);
    const uint32_t threads = tu.block_threads;
    const uint64_t waves_needed = ((uint64_t)w.nq + 63) / 64;
    uint64_t blocks = (uint64_t)di.num_cus * tu.blocks_per_cu;
    const uint64_t max_useful = (waves_needed * 64 + threads - 1) / threads;
    if (blocks > max_useful) blocks = max_useful;
    if (blocks == 0) blocks = 1;
    switch (tu.walkers_per_lane) {
        case 2:
            hipLaunchKernelGGL((k_walk_persistent<ALGO, SMP, 2>), dim3(blocks), dim3(threads), 0, s, g, t, w, head, tu.queue_chunk);
            break;
        case 4:
            hipLaunchKernelGGL((k_walk_persistent<ALGO, SMP, 4>), dim3(blocks), dim3(threads), 0, s, g, t, w, head, tu.queue_chunk);
            break;
        default:
            hipLaunchKernelGGL((k_walk_persistent<ALGO, SMP, 1>), dim3(blocks), dim3(threads), 0, s, g, t, w, head, tu.queue_chunk);
    }
    return hipGetLastError();
}

template <uint32_t ALGO, uint32_t SMP>
hipError_t run_bsp(const GraphDev &g, const TableDev &t, const WalkDev &w, const Tuning &tu,
                   const DeviceInfo &di, void *ws, hipStream_t s) {
    constexpr bool kAlias = (SMP == SMP_ALIAS) && (ALGO == ALG_DEEPWALK || ALGO == ALG_PPR);
    char *base = reinterpret_cast<char *>(ws);
    uint32_t *counts = reinterpret_cast<uint32_t *>(base);
    const size_t counts_bytes = round_up(sizeof(uint32_t) * (w.max_len + 2));
    Rec *lists[2] = {reinterpret_cast<Rec *>(base + counts_bytes),
                     reinterpret_cast<Rec *>(base + counts_bytes + round_up(sizeof(Rec) * (size_t)w.nq))};
    const uint32_t nfill = w.max_len + 2;
    hipLaunchKernelGGL(k_fill_u32, dim3((nfill + 255) / 256), dim3(256), 0, s, counts, nfill, 0u);
    const uint32_t threads = tu.block_threads;
    uint64_t blocks = (uint64_t)di.num_cus * tu.blocks_per_cu;
    const uint64_t need = ((uint64_t)w.nq + threads - 1) / threads;
    if (blocks > need) blocks = need;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_bsp_init<kAlias>, dim3(blocks), dim3(threads), 0, s, g, w, lists[0], counts);
    for (uint32_t k = 0; k < w.max_len; ++k) {
        hipLaunchKernelGGL((k_bsp_step<ALGO, SMP>), dim3(blocks), dim3(threads), 0, s, g, t, w, k,
                           lists[k & 1], counts + k, lists[(k + 1) & 1], counts + k + 1);
    }
    return hipGetLastError();
}

template <uint32_t ALGO, uint32_t SMP>
hipError_t run(const GraphDev &g, const TableDev &t, const WalkDev &w, uint32_t mode, const Tuning &tu,
               const DeviceInfo &di, void *ws, hipStream_t s) {
    return mode == TRW_M_PERSISTENT ? run_persistent<ALGO, SMP>(g, t, w, tu, di, ws, s)
                                    : run_bsp<ALGO, SMP>(g, t, w, tu, di, ws, s);
}

}  // namespace

size_t walk_workspace_bytes(uint32_t mode, uint64_t nq, uint32_t max_len) {
    if (mode == TRW_M_PERSISTENT) return kAlign;
    return round_up(sizeof(uint32_t) * (max_len + 2)) + 2 * round_up(sizeof(Rec) * (size_t)nq);
}

hipError_t launch_walk(const GraphDev &g, const TableDev &t, uint32_t algo, uint32_t sampler,
                       const WalkDev &w, uint32_t mode, const Tuning &tu, const DeviceInfo &di,
                       void *ws, size_t, hipStream_t s) {
    if (w.nq == 0) return hipSuccess;
    switch (algo) {
        case ALG_DEEPWALK:
            if (sampler == SMP_NAIVE) return run<ALG_DEEPWALK, SMP_NAIVE>(g, t, w, mode, tu, di, ws, s);
            if (sampler == SMP_ALIAS) return run<ALG_DEEPWALK, SMP_ALIAS>(g, t, w, mode, tu, di, ws, s);
            return run<ALG_DEEPWALK, SMP_ITS>(g, t, w, mode, tu, di, ws, s);
        case ALG_PPR:
            if (sampler == SMP_NAIVE) return run<ALG_PPR, SMP_NAIVE>(g, t, w, mode, tu, di, ws, s);
            if (sampler == SMP_ALIAS) return run<ALG_PPR, SMP_ALIAS>(g, t, w, mode, tu, di, ws, s);
            return run<ALG_PPR, SMP_ITS>(g, t, w, mode, tu, di, ws, s);
        case ALG_NODE2VEC:
            return run<ALG_NODE2VEC, SMP_OREJ>(g, t, w, mode, tu, di, ws, s);
        default:
            return run<ALG_METAPATH, SMP_ITS>(g, t, w, mode, tu, di, ws, s);
    }
}

}  // namespace trw
