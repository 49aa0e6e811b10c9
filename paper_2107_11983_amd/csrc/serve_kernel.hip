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

// Wave-uniform values kept in scalar registers.
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long uniform64(unsigned long long v) {
    return ((unsigned long long)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

// A query ended: its length and status go to its request's outputs; the
// request's completion count is added to by count_done, once per wave and
// request.
__device__ __forceinline__ void finish(const ReqRegs &q, SlotState &st, uint8_t status, uint32_t &fin_req) {
    q.lengths[st.qi] = st.k;
    q.status[st.qi] = status;
    fin_req = st.req;
    st.req = kIdle;
}

// Wave-uniform: the queries that ended since the last call, added to their
// requests' completion counters with one atomic per distinct request.
__device__ __forceinline__ void count_done(const ServeDev &s, uint32_t &fin_req) {
    uint64_t todo = __ballot(fin_req != kIdle);
    while (todo != 0) {
        const int leader = (int)__builtin_ctzll(todo);
        const uint32_t r = __shfl(fin_req, leader);
        const uint64_t same = __ballot(fin_req == r);
        if (lane_id() == (uint32_t)leader) atomicAdd(&s.done[r], (uint32_t)__popcll(same));
        todo &= ~same;
    }
    fin_req = kIdle;
}

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

// Lane i's query of chunk [begin, end) of request req: its source (the row
// range follows once the source has arrived).
__device__ __forceinline__ int32_t chunk_source(const ServeDev &s, uint32_t req, uint32_t begin, uint32_t end) {
    const uint32_t qi = begin + lane_id();
    return qi < end ? s.reqs[req].sources[qi] : -1;
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
    PathBuf path;
    ReqRegs q;
    if (st.req != kIdle) {
        load_req(s.reqs[st.req], q);
        path.start(path_entry(s, st.req, st.qi, st.k + 1));
    }
    uint32_t moves = 0;
    uint32_t fin_req = kIdle;

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
            if (((idle >> lane) & 1ull) && rk < avail) {
                load_req(s.reqs[ws.req], q);
                st.req = ws.req; st.qi = ws.next + rk; st.k = 0; st.prev = -1; st.poff = 0; st.pdeg = 0;
                if (src < 0 || src >= g.n) {
                    finish(q, st, ST_BAD_SOURCE, fin_req);
                } else if (deg == 0 || q.cancelled) {
                    *path_entry(s, st.req, st.qi, 0) = src;
                    if (q.cancelled) { fin_req = st.req; st.req = kIdle; }   // counted, no outputs
                    else finish(q, st, ST_DEAD_END, fin_req);
                } else {
                    st.cur = src; st.off = off; st.deg = deg;
                    path.start(path_entry(s, st.req, st.qi, 0));
                    path.push(src);
                }
            }
            ws.next = uniform(ws.next + min((uint32_t)__popcll(idle), avail));
            count_done(s, fin_req);
            idle = __ballot(st.req == kIdle);
        }
        // The following chunk, loaded ahead: its rows once its sources are in,
        // or a new one from the ring.
        int32_t b_hi = 0;
        bool b_rows = false;
        if (b_stage == 1) {
            chunk_rows(g, b, b_hi);
            b_rows = true;
            b_stage = 2;
        } else if (ws.n_end == ws.n_begin) {
            if (!ws.has_claim) {
                unsigned long long c = 0;
                if (lane == 0) c = atomicAdd(s.head, 1ull);
                ws.claim = uniform64(__shfl(c, 0));
                ws.has_claim = 1;
            }
            if (ws.claim < tail) {                       // published: take it
                const Chunk ch = s.ring[ws.claim % s.ring_size];
                ws.n_req = uniform(ch.req); ws.n_begin = uniform(ch.begin); ws.n_end = uniform(ch.end);
                ws.has_claim = 0;
                b.src = chunk_source(s, ws.n_req, ws.n_begin, ws.n_end);
                b_stage = 1;
            }
        }
        if (__ballot(st.req != kIdle) == 0) {
            if (ws.n_end == ws.n_begin) break;         // nothing to run: the ring is drained for now
            continue;                                  // the chunk just taken starts in the next iteration
        }

        // Move.
        int32_t nxt = -1, noff = 0, ndeg = 0;
        Rand4 r{};
        const bool walking = st.req != kIdle && !q.cancelled;
        if (walking) {
            const uint64_t qid = q.qid_base + st.qi;
            r = philox(st.k, 0, qid, q.wd.seed);
            if (st.deg != 0) {
                if (q.algo == ALG_NODE2VEC) {
                    if (t.adj) {
                        nxt = n2v_move<true>(g, t, q.wd, qid, st.k, st.off, (uint32_t)st.deg, r, st.prev, st.poff,
                                             st.pdeg, noff, ndeg);
                    } else {
                        nxt = n2v_move<false>(g, t, q.wd, qid, st.k, st.off, (uint32_t)st.deg, r, st.prev, st.poff,
                                              st.pdeg, noff, ndeg);
                        if (nxt >= 0) { noff = g.row_ptr[nxt]; ndeg = g.row_ptr[nxt + 1] - noff; }
                    }
                } else if (q.sampler == SMP_ALIAS) {
                    const uint32_t e = (uint32_t)st.off + scale32(r.r0, (uint32_t)st.deg);
                    nxt = alias_pick(t.alias[2 * (uint64_t)e], t.alias[2 * (uint64_t)e + 1], r.r1, noff, ndeg);
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
        }
        // The following chunk's loads were issued before the move's reads and
        // have arrived with them; the empty asm uses them here on every path
        // through the loop, not at the top of the next iteration.
        asm volatile("" ::"v"(b.src), "v"(b.off), "v"(b_hi));
        if (b_rows) b.deg = b_hi - b.off;

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
        count_done(s, fin_req);
    }
    path.flush();
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
