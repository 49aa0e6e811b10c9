// Serving tick: one launch advances every walker slot of the server by up to
// `steps` moves.  Slots whose walk ends take the next query of their wave's
// current chunk; chunks (up to 64 queries of one request) come from a FIFO
// ring that the host fills as it admits requests, so requests admitted while
// others run share the device from the next tick on (continuous batching).
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

// The fields of a walker's request that every step needs, held in registers
// (the descriptor table only changes between ticks).
struct ReqRegs {
    uint32_t algo, sampler, max_len, stop_q32, cancelled;
    WalkDev wd;              // thresholds and seed in the layout the move functions take
    uint64_t qid_base;
    int32_t *paths;
    uint64_t stride;
    uint32_t *lengths;
    uint8_t *status;
};

__device__ __forceinline__ void load_req(const ReqDesc &d, ReqRegs &q) {
    q.algo = d.algo; q.sampler = d.sampler; q.max_len = d.max_len; q.stop_q32 = d.stop_q32;
    q.cancelled = d.cancelled;
    q.wd.thr[0] = d.thr[0]; q.wd.thr[1] = d.thr[1]; q.wd.thr[2] = d.thr[2];
    q.wd.seed = d.seed;
    q.qid_base = d.qid_base;
    q.paths = d.paths; q.stride = d.stride; q.lengths = d.lengths; q.status = d.status;
}

__device__ __forceinline__ void finish(const ServeDev &s, const ReqRegs &q, SlotState &st, uint8_t status) {
    q.lengths[st.qi] = st.k;
    q.status[st.qi] = status;
    atomicAdd(&s.done[st.req], 1u);
    st.req = kIdle;
}

__global__ void __launch_bounds__(256) k_serve_tick(GraphDev g, TableDev t, ServeDev s, uint32_t steps) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t wid = gid >> 6;
    const uint32_t lane = lane_id();
    SlotState st = s.slots[gid];
    WaveState ws = s.waves[wid];                       // same value in every lane
    const unsigned long long tail = *s.tail;           // chunks published before this tick
    PathBuf path;
    ReqRegs q;
    if (st.req != kIdle) {
        load_req(s.reqs[st.req], q);
        path.start(q.paths + (uint64_t)st.qi * q.stride + st.k + 1);
    }
    uint32_t moves = 0;

    for (uint32_t it = 0; it < steps; ++it) {
        // Refill idle slots from the wave's chunk, claiming chunks in ring order.
        uint64_t idle = __ballot(st.req == kIdle);
        while (idle != 0) {
            if (ws.next == ws.end) {
                if (!ws.has_claim) {
                    unsigned long long c = 0;
                    if (lane == 0) c = atomicAdd(s.head, 1ull);
                    ws.claim = __shfl(c, 0);
                    ws.has_claim = 1;
                }
                if (ws.claim >= tail) break;          // not published yet: keep the claim
                const Chunk ch = s.ring[ws.claim % s.ring_size];
                ws.req = ch.req; ws.next = ch.begin; ws.end = ch.end; ws.has_claim = 0;
            }
            const uint32_t avail = ws.end - ws.next;
            const uint32_t rk = rank_below(idle);
            if (((idle >> lane) & 1ull) && rk < avail) {
                const ReqDesc &d = s.reqs[ws.req];
                load_req(d, q);
                st.req = ws.req;
                st.qi = ws.next + rk;
                st.k = 0;
                st.prev = -1;
                st.poff = 0; st.pdeg = 0;
                const int32_t src = d.sources[st.qi];
                if (src < 0 || src >= g.n) {
                    finish(s, q, st, ST_BAD_SOURCE);
                } else {
                    st.cur = src;
                    const int32_t lo = g.row_ptr[src];
                    st.off = lo;
                    st.deg = g.row_ptr[src + 1] - lo;
                    path.start(q.paths + (uint64_t)st.qi * q.stride);
                    path.push(src);
                }
            }
            ws.next += min((uint32_t)__popcll(idle), avail);
            idle = __ballot(st.req == kIdle);
        }
        if (__ballot(st.req != kIdle) == 0) break;     // nothing to run this tick

        if (st.req != kIdle) {
            if (q.cancelled) {
                path.flush();
                atomicAdd(&s.done[st.req], 1u);
                st.req = kIdle;
                continue;
            }
            const uint64_t qid = q.qid_base + st.qi;
            const Rand4 r = philox(st.k, 0, qid, q.wd.seed);
            int32_t nxt = -1, noff = 0, ndeg = 0;
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
            if (nxt < 0) {
                path.flush();
                finish(s, q, st, ST_DEAD_END);
                continue;
            }
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
                finish(s, q, st, status);
            }
        }
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
