// Serving tick: one launch advances every walker slot of the server by up to
// `steps` moves.  Slots whose walk ends start the next query of their wave's
// current chunk, whose sources and row ranges the wave loaded ahead; chunks
// (up to 64 queries of one request) come from a FIFO ring that the host fills
// as it admits requests, so requests admitted while others run share the
// device from the next tick on (continuous batching).
// Walker state lives in device memory between ticks; the launch shape never
// changes, so the host captures the tick once as a graph and replays it.
//
// A query's walk depends only on its request's parameters, seed and
// qid = qid_base + index: the same request gives the same paths alone, in any
// mix, and through trw_walk.
#include "serve_internal.hpp"
#include "trw_device.hpp"
#include "walk_common.hpp"

namespace trw {
namespace {

// The fields of a walker's request that its moves and its end need, held in
// registers (the descriptor table only changes between ticks).  The path row
// is located once, when the walk starts (or a tick resumes it).
struct ReqRegs {
    uint32_t algo, sampler, max_len, stop_q32, cancelled;
    WalkDev wd;              // thresholds and seed in the layout the move functions take
    uint64_t qid_base;
    uint32_t *lengths;
    uint8_t *status;
};

// The descriptor of request slot r when r is the same in every lane: the
// table does not change during a tick, so it is read through the constant
// address space (scalar loads).  A wait for scalar loads does not wait for
// the vector stores still in flight, as a wait for vector loads does.
__device__ __forceinline__ ReqDesc desc_uniform(const ServeDev &s, uint32_t r) {
    const auto &c = ((const __attribute__((address_space(4))) ReqDesc *)s.reqs)[r];
    ReqDesc d;
    d.algo = c.algo; d.sampler = c.sampler; d.max_len = c.max_len; d.stop_q32 = c.stop_q32;
    d.thr[0] = c.thr[0]; d.thr[1] = c.thr[1]; d.thr[2] = c.thr[2];
    d.cancelled = c.cancelled;
    d.seed = c.seed; d.qid_base = c.qid_base;
    d.sources = c.sources; d.paths = c.paths; d.lengths = c.lengths; d.status = c.status;
    d.stride = c.stride; d.nq = c.nq; d.pad = 0;
    return d;
}

// Ring entry i, read the same way (published by the host before the tick).
__device__ __forceinline__ Chunk ring_uniform(const ServeDev &s, unsigned long long i) {
    const auto &c = ((const __attribute__((address_space(4))) Chunk *)s.ring)[i % s.ring_size];
    Chunk ch;
    ch.req = c.req; ch.begin = c.begin; ch.end = c.end; ch.pad = 0;
    return ch;
}

__device__ __forceinline__ void load_req(const ReqDesc &d, ReqRegs &q) {
    q.algo = d.algo; q.sampler = d.sampler; q.max_len = d.max_len; q.stop_q32 = d.stop_q32;
    q.cancelled = d.cancelled;
    q.wd.thr[0] = d.thr[0]; q.wd.thr[1] = d.thr[1]; q.wd.thr[2] = d.thr[2];
    q.wd.seed = d.seed;
    q.wd.n2v_search = 0;     // Node2Vec's adjacency test probes the edge index's hash set for every row
    q.qid_base = d.qid_base;
    q.lengths = d.lengths; q.status = d.status;
}

// Entry `k` of query qi's path row in request slot req.
__device__ __forceinline__ int32_t *path_entry(const ServeDev &s, uint32_t req, uint32_t qi, uint32_t k) {
    const ReqDesc &d = s.reqs[req];
    return d.paths + (uint64_t)qi * d.stride + k;
}

// Lane 0's value of a 64-bit register, in scalar registers.
__device__ __forceinline__ unsigned long long lane0_64(unsigned long long v) {
    return ((unsigned long long)__builtin_amdgcn_readlane((uint32_t)(v >> 32), 0) << 32) |
           __builtin_amdgcn_readlane((uint32_t)v, 0);
}

// Wave-uniform values kept in scalar registers.
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long uniform64(unsigned long long v) {
    return ((unsigned long long)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

// A query ended: its length and status go to its request's outputs; the
// request's completion count is added to by count_done.
__device__ __forceinline__ void finish(const ReqRegs &q, SlotState &st, uint8_t status, uint32_t &fin_req) {
    global_ptr(q.lengths)[st.qi] = st.k;
    global_ptr(q.status)[st.qi] = status;
    fin_req = st.req;
    st.req = kIdle;
}

// Queries ended during the tick, per wave and request: the counts of up to
// four requests are kept in scalar registers and added to the requests'
// completion counters when the tick ends (the host reads them only between
// ticks); a fifth request ended in the same tick is added at once.  So a wave
// makes no atomic per iteration, and a move's wait for its read does not wait
// for atomics held up on a counter that many waves add to.
struct DoneCounts {
    uint32_t r0, r1, r2, r3;
    uint32_t c0, c1, c2, c3;
    uint32_t n;
};

__device__ __forceinline__ void count_done(const ServeDev &s, uint32_t &fin_req, DoneCounts &d) {
    uint64_t todo = __ballot(fin_req != kIdle);
    while (todo != 0) {
        const int leader = (int)__builtin_ctzll(todo);
        const uint32_t r = __builtin_amdgcn_readlane(fin_req, leader);
        const uint64_t same = __ballot(fin_req == r);
        const uint32_t k = (uint32_t)__popcll(same);
        if (d.n > 0 && d.r0 == r) d.c0 += k;
        else if (d.n > 1 && d.r1 == r) d.c1 += k;
        else if (d.n > 2 && d.r2 == r) d.c2 += k;
        else if (d.n > 3 && d.r3 == r) d.c3 += k;
        else if (d.n == 0) { d.r0 = r; d.c0 = k; d.n = 1; }
        else if (d.n == 1) { d.r1 = r; d.c1 = k; d.n = 2; }
        else if (d.n == 2) { d.r2 = r; d.c2 = k; d.n = 3; }
        else if (d.n == 3) { d.r3 = r; d.c3 = k; d.n = 4; }
        else if (lane_id() == (uint32_t)leader) atomicAdd(&s.done[r], k);
        todo &= ~same;
    }
    fin_req = kIdle;
}

__device__ __forceinline__ void flush_done(const ServeDev &s, const DoneCounts &d) {
    if (lane_id() == 0) {
        if (d.n > 0) atomicAdd(&s.done[d.r0], d.c0);
        if (d.n > 1) atomicAdd(&s.done[d.r1], d.c1);
        if (d.n > 2) atomicAdd(&s.done[d.r2], d.c2);
        if (d.n > 3) atomicAdd(&s.done[d.r3], d.c3);
    }
}

// The tick's path writer: up to 4 pending entries per walker, written as one
// 16-byte store when they end on a 16-byte boundary, else entry by entry (the
// batch walker's rules), every store made through a global pointer.
struct TickPath {
    int32_t *p;      // address of the first pending entry
    uint32_t n;      // pending entries
    int32_t b0, b1, b2, b3;

    __device__ __forceinline__ void start(int32_t *row) { p = row; n = 0; }

    __device__ __forceinline__ void flush() {
        if (n == 4) {
            auto *q = global_ptr(static_cast<int32_t *>(__builtin_assume_aligned(p, 16)));
            q[0] = b0; q[1] = b1; q[2] = b2; q[3] = b3;
        } else {
            auto *q = global_ptr(p);
            if (n > 0) q[0] = b0;
            if (n > 1) q[1] = b1;
            if (n > 2) q[2] = b2;
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

// Query starts prepared ahead, one query per lane: lane i holds the source
// and row range of query begin + i of the wave's current chunk (a_*) and of
// query n_begin + i of the following chunk (b_*).  A walker that ends takes
// the next unstarted query's values from the lane holding them (a lane
// shuffle), so a start waits for no load, and a query whose source has no
// edges (or is out of range) ends in the refill loop itself.  Queries stay
// with their wave, never with a busy lane, until a lane is free to run them.
struct Prepared {
    int32_t src, off, deg;
};

// Lane i's query of chunk [begin, end) of request req (wave-uniform): its
// source (the row range follows once the source has arrived).
__device__ __forceinline__ int32_t chunk_source(const ServeDev &s, uint32_t req, uint32_t begin, uint32_t end) {
    const int32_t *src = desc_uniform(s, req).sources;
    const uint32_t qi = begin + lane_id();
    return qi < end ? global_ptr(src)[qi] : -1;
}

__device__ __forceinline__ void chunk_rows(const GraphDev &g, Prepared &p, int32_t &hi) {
    if (p.src >= 0 && p.src < g.n) {
        p.off = g.row_ptr[p.src];
        hi = g.row_ptr[p.src + 1];
    } else {
        p.off = 0;
        hi = 0;
    }
}

__global__ void __launch_bounds__(256) k_serve_tick(GraphDev g, TableDev t, ServeDev s, uint32_t steps) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t wid = gid >> 6;
    const uint32_t lane = lane_id();
    SlotState st = s.slots[gid];
    WaveState ws = s.waves[wid];                       // same value in every lane
    ws.claim = uniform64(ws.claim); ws.has_claim = uniform(ws.has_claim);
    ws.req = uniform(ws.req); ws.begin = uniform(ws.begin); ws.next = uniform(ws.next); ws.end = uniform(ws.end);
    ws.n_req = uniform(ws.n_req); ws.n_begin = uniform(ws.n_begin); ws.n_end = uniform(ws.n_end);
    const unsigned long long tail = *s.tail;           // chunks published before this tick

    // The prepared values of both chunks are reloaded at the start of a tick.
    Prepared a{-1, 0, 0}, b{-1, 0, 0};
    uint32_t b_stage = 0;                              // following chunk: 1 sources loading, 2 rows loading or ready
    {
        int32_t a_hi = 0, b_hi = 0;
        if (ws.next != ws.end) a.src = chunk_source(s, ws.req, ws.begin, ws.end);
        if (ws.n_end != ws.n_begin) { b.src = chunk_source(s, ws.n_req, ws.n_begin, ws.n_end); b_stage = 2; }
        if (ws.next != ws.end) { chunk_rows(g, a, a_hi); a.deg = a_hi - a.off; }
        if (b_stage) { chunk_rows(g, b, b_hi); b.deg = b_hi - b.off; }
    }
    TickPath path;
    ReqRegs q;
    if (st.req != kIdle) {
        load_req(s.reqs[st.req], q);
        path.start(path_entry(s, st.req, st.qi, st.k + 1));
    }
    uint32_t moves = 0;
    uint32_t fin_req = kIdle;
    DoneCounts dc{0, 0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long c_pend = 0;                     // lane 0: a claim's atomic, issued, not yet read
    bool claim_issued = false;
    // Every load above has arrived before the loop: one left outstanding
    // would be waited for inside the loop, and that wait, repeated in each
    // iteration, would also wait for the stores of the iteration before.
    __builtin_amdgcn_s_waitcnt(0);

    for (uint32_t it = 0; it < steps; ++it) {
        // Refill: idle lanes start the current chunk's next queries.
        uint64_t idle = __ballot(st.req == kIdle);
        while (idle != 0) {
            if (ws.next == ws.end) {
                if (ws.n_end == ws.n_begin) break;     // no following chunk yet
                if (b_stage == 1) {                      // its rows were not requested yet: do it now
                    int32_t hi = 0;
                    chunk_rows(g, b, hi);
                    b.deg = hi - b.off;
                }
                a = b;
                ws.req = ws.n_req; ws.begin = ws.n_begin; ws.next = ws.n_begin; ws.end = ws.n_end;
                ws.n_begin = ws.n_end = 0;
                b_stage = 0;
            }
            const uint32_t avail = ws.end - ws.next;
            const uint32_t rk = rank_below(idle);
            const int j = (int)min(ws.next - ws.begin + rk, 63u);
            const int32_t src = __shfl(a.src, j), off = __shfl(a.off, j), deg = __shfl(a.deg, j);
            const ReqDesc dq = desc_uniform(s, ws.req);
            if (((idle >> lane) & 1ull) && rk < avail) {
                load_req(dq, q);
                st.req = ws.req; st.qi = ws.next + rk; st.k = 0; st.prev = -1; st.poff = 0; st.pdeg = 0;
                int32_t *row = dq.paths + (uint64_t)st.qi * dq.stride;
                if (src < 0 || src >= g.n) {
                    finish(q, st, ST_BAD_SOURCE, fin_req);
                } else if (deg == 0 || q.cancelled) {
                    *global_ptr(row) = src;
                    if (q.cancelled) { fin_req = st.req; st.req = kIdle; }   // counted, no outputs
                    else finish(q, st, ST_DEAD_END, fin_req);
                } else {
                    st.cur = src; st.off = off; st.deg = deg;
                    path.start(row);
                    path.push(src);
                }
            }
            ws.next = uniform(ws.next + min((uint32_t)__popcll(idle), avail));
            count_done(s, fin_req, dc);
            idle = __ballot(st.req == kIdle);
        }
        // The following chunk, loaded ahead: its rows once its sources are in,
        // or a new one from the ring.  Loads go to temporaries that are
        // committed to the loop's state only after this iteration has waited
        // for them (after the move's reads, or on the path with no move), so
        // no load is outstanding at the bottom of the loop: a wait there would
        // also wait for the iteration's stores.
        int32_t n_src = 0, n_off = 0, n_hi = 0;
        unsigned long long c_new = 0;
        bool took = false, rows = false, issued = false;
        if (b_stage == 1) {
            if (b.src >= 0 && b.src < g.n) {
                n_off = g.row_ptr[b.src];
                n_hi = g.row_ptr[b.src + 1];
            }
            rows = true;
            b_stage = 2;
        } else if (ws.n_end == ws.n_begin) {
            if (claim_issued) {                          // a claim made in an earlier iteration
                ws.claim = lane0_64(c_pend);
                ws.has_claim = 1;
                claim_issued = false;
            }
            if (!ws.has_claim) {
                if (lane == 0) c_new = atomicAdd(s.head, 1ull);
                issued = true;
            } else if (ws.claim < tail) {                // published: take it
                const Chunk ch = ring_uniform(s, ws.claim);
                ws.n_req = uniform(ch.req); ws.n_begin = uniform(ch.begin); ws.n_end = uniform(ch.end);
                ws.has_claim = 0;
                n_src = chunk_source(s, ws.n_req, ws.n_begin, ws.n_end);
                took = true;
                b_stage = 1;
            }
        }
        auto commit = [&]() {
            asm volatile("" ::"v"(n_src), "v"(n_off), "v"(n_hi), "v"(c_new));
            if (took) b.src = n_src;
            if (rows) { b.off = n_off; b.deg = n_hi - n_off; }
            if (issued) { c_pend = c_new; claim_issued = true; }
        };
        if (__ballot(st.req != kIdle) == 0) {
            // nothing to run and nothing coming: the ring is drained for now
            if (ws.n_end == ws.n_begin && !issued && !(ws.has_claim && ws.claim < tail)) break;
            commit();                                  // a chunk taken or claimed starts later
            continue;
        }

        // Move.  The first read of every walking lane is issued before any
        // lane waits: the 32-byte ALIAS entry, or the adjacency record of a
        // Node2Vec walker's first dart (same slot formula).  Lanes of both
        // kinds in one wave then wait once, not once per kind.
        int32_t nxt = -1, noff = 0, ndeg = 0;
        Rand4 r{};
        const bool walking = st.req != kIdle && !q.cancelled;
        const bool n2v_adj = q.algo == ALG_NODE2VEC && t.adj != nullptr;
        uint4 A = make_uint4(0, 0, 0, 0), B = make_uint4(0, 0, 0, 0);
        if (walking) {
            const uint64_t qid = q.qid_base + st.qi;
            r = philox(st.k, 0, qid, q.wd.seed);
            if (st.deg != 0) {
                const uint32_t e = (uint32_t)st.off + scale32(r.r0, (uint32_t)st.deg);
                if (n2v_adj) {
                    A = t.adj[e];
                } else if (q.algo != ALG_NODE2VEC && q.sampler == SMP_ALIAS) {
                    A = t.alias[2 * (uint64_t)e];
                    B = t.alias[2 * (uint64_t)e + 1];
                }
            }
        }
        asm volatile("" ::"v"(A.x), "v"(A.y), "v"(A.z), "v"(B.x), "v"(B.y), "v"(B.z), "v"(B.w));
        if (walking && st.deg != 0) {
            const uint64_t qid = q.qid_base + st.qi;
            if (q.algo == ALG_NODE2VEC) {
                if (n2v_adj) {
                    nxt = n2v_move<true, true>(g, t, q.wd, qid, st.k, st.off, (uint32_t)st.deg, r, st.prev, st.poff,
                                               st.pdeg, noff, ndeg, A);
                } else {
                    nxt = n2v_move<false>(g, t, q.wd, qid, st.k, st.off, (uint32_t)st.deg, r, st.prev, st.poff,
                                          st.pdeg, noff, ndeg);
                    if (nxt >= 0) { noff = g.row_ptr[nxt]; ndeg = g.row_ptr[nxt + 1] - noff; }
                }
            } else if (q.sampler == SMP_ALIAS) {
                nxt = alias_pick(A, B, r.r1, noff, ndeg);
            } else {  // NAIVE
                const uint32_t e = (uint32_t)st.off + scale32(r.r0, (uint32_t)st.deg);
                if (t.adj) {
                    const uint4 rec = t.adj[e];
                    nxt = (int32_t)rec.x; noff = (int32_t)rec.y; ndeg = (int32_t)rec.z;
                } else {
                    nxt = g.col[e];
                    noff = g.row_ptr[nxt]; ndeg = g.row_ptr[nxt + 1] - noff;
                }
            }
        }
        // The following chunk's loads were issued before the move's reads and
        // have arrived with them.
        commit();

        // Update.
        if (st.req != kIdle && q.cancelled) {          // counted, no outputs
            path.flush();
            fin_req = st.req;
            st.req = kIdle;
        } else if (walking) {
            if (nxt < 0) {
                path.flush();
                finish(q, st, ST_DEAD_END, fin_req);
            } else {
                path.push(nxt);
                ++moves;
                st.prev = st.cur; st.poff = st.off; st.pdeg = st.deg;
                st.cur = nxt; st.off = noff; st.deg = ndeg;
                st.k += 1;
                uint8_t status = 0;
                if (q.algo == ALG_PPR && r.r2 < q.stop_q32) status = ST_STOPPED;
                else if (st.k == q.max_len) status = ST_LENGTH;
                if (status) {
                    path.flush();
                    finish(q, st, status, fin_req);
                }
            }
        }
        count_done(s, fin_req, dc);
    }
    path.flush();
    if (claim_issued) {
        ws.claim = lane0_64(c_pend);
        ws.has_claim = 1;
    }
    flush_done(s, dc);
    s.slots[gid] = st;
    if (lane == 0) s.waves[wid] = ws;
    const uint32_t wave_moves = wave_total(moves);
    if (lane == 0 && wave_moves) atomicAdd(s.moves, (unsigned long long)wave_moves);
}

}  // namespace

hipError_t launch_serve_tick(const GraphDev &g, const TableDev &t, const ServeDev &s, uint32_t steps,
                             uint32_t blocks, hipStream_t stream) {
    hipLaunchKernelGGL(k_serve_tick, dim3(blocks), dim3(kServeBlock), 0, stream, g, t, s, steps);
    return hipGetLastError();
}

}  // namespace trw
