// Serving: a resident graph and tables, a fixed pool of walker slots on the
// device, and a host thread that admits requests, publishes their queries in
// chunks and replays the tick graph while anything is in flight.
//
// Memory: one caller-provided arena holds the fixed device state (request
// descriptors, chunk ring, counters, walker slots) followed by a pool.  A
// request with device buffers is read and written in place and takes no pool
// space; one with host buffers gets its input copy and output rows from the
// pool.  A request waits (first come, first served) until a descriptor slot
// and pool space are free; one that could never fit is refused at submit.
//
// Per tick the thread (1) admits what fits and publishes the descriptor table
// and the new ring chunks (one copy each), (2) launches the tick (a captured
// graph), (3) reads all completion counters back in one copy, and (4)
// completes the requests that finished: device outputs are already in place,
// host outputs are copied out of the pool.  The host cost per tick is a fixed
// handful of calls, whatever the number of requests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "serve_internal.hpp"
#include "trw_internal.hpp"

namespace trw {

__global__ void k_fill_bytes(uint32_t *p, size_t n_words, uint32_t v) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += stride) p[i] = v;
}

// A 2D copy of `rows` rows of `width` bytes (host outputs of a finished request).
struct CopyJob {
    const char *src;
    char *dst;
    uint64_t src_pitch, dst_pitch, width, rows;
};

namespace {

constexpr size_t kA = 256;
inline size_t align_up(size_t x) { return (x + kA - 1) / kA * kA; }

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over [0, size) with coalescing of free ranges.
class RangeAllocator {
  public:
    explicit RangeAllocator(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

  private:
    size_t size_;
    size_t used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Layout {
    size_t reqs, ring, counters, done, done_bytes, slots, waves, pool, fixed;
};

// The completion counters are followed by the moves counter so that one copy
// brings both back.
Layout layout(uint32_t slots, uint32_t max_reqs, uint32_t ring) {
    Layout l{};
    size_t o = 0;
    l.reqs = o; o = align_up(o + sizeof(ReqDesc) * max_reqs);
    l.ring = o; o = align_up(o + sizeof(Chunk) * ring);
    l.counters = o; o = align_up(o + 2 * sizeof(unsigned long long));   // head, tail
    l.done = o;
    l.done_bytes = (sizeof(uint32_t) * max_reqs + 7) / 8 * 8 + sizeof(unsigned long long);
    o = align_up(o + l.done_bytes);
    l.slots = o; o = align_up(o + sizeof(SlotState) * slots);
    l.waves = o; o = align_up(o + sizeof(WaveState) * (slots / 64));
    l.pool = o;
    l.fixed = o;
    return l;
}

struct Pending {
    uint64_t id;
    trw_request req;
    uint64_t t_submit;
    size_t bytes;
};

struct Active {
    uint64_t id;
    trw_request req;
    uint64_t t_submit, t_admit;
    size_t pool_off, pool_bytes;
    unsigned long long first_chunk;   // ring index of the request's first chunk
    uint32_t slot;
    uint32_t done_base;        // the slot's completion counter when this request was admitted
    uint64_t stride;
    size_t out_off;            // offset of the outputs inside the request's pool range
    bool finishing = false;
    bool cancelled = false;
    uint64_t batch_seq = 0;    // the delivery batch it finished in (when finishing)
};

// Mark descriptor slot i as changed (copied to the device before the next tick).
void desc_touch(trw_server_s *s, uint32_t i);

// The requests that finished in one tick.  Host outputs are copied on the
// delivery stream; the requests complete when `done` has been reached (no
// event when the batch had nothing to copy).
struct Batch {
    hipEvent_t done = nullptr;
    uint64_t seq = 0;                  // its sequence number (Active::batch_seq of its requests)
    std::vector<uint64_t> ids;
};

}  // namespace
}  // namespace trw

using namespace trw;

struct trw_server_s {
    // configuration
    GraphDev g;
    TableDev t;
    uint32_t slots, max_reqs, ring, steps;
    bool use_graph;
    bool pipelined;
    int device;
    // device memory
    char *arena;
    Layout lay;
    ServeDev dev;
    RangeAllocator pool;
    // host staging (pinned).  Ticks are pipelined one deep: while tick i runs
    // the host reads tick i-1's counters and completes its finished requests
    // (host outputs copied on a second stream), so the tail and the counter
    // read-back have two halves, used by alternate ticks.
    ReqDesc *h_desc = nullptr;                // mirror of the device descriptor table
    Chunk *h_ring = nullptr;
    unsigned long long *h_tail = nullptr;     // [2]
    uint32_t *h_done = nullptr;               // [2] x (completion counters, then the moves counter)
    uint32_t desc_lo = 0, desc_hi = 0;        // descriptor slots changed since the last copy: [lo, hi)
    hipStream_t stream = nullptr;             // ticks and the copies that feed them
    hipStream_t deliver_stream = nullptr;     // host output copies of finished requests
    hipEvent_t tick_done[2] = {nullptr, nullptr};
    hipEvent_t tick_start[2] = {nullptr, nullptr};
    hipEvent_t tick_end[2] = {nullptr, nullptr};     // right after the tick kernel, before the read-back
    std::deque<Batch> batches;
    std::vector<hipEvent_t> spare_events;
    uint64_t n_batches = 0;
    std::vector<uint32_t> slot_done;          // a request slot's completion counter once all its requests ended
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // scheduling state (guarded by mu)
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> waiting;
    std::vector<uint64_t> cancel_requests;
    std::deque<trw_completion> completed;
    bool stopping = false;
    uint64_t next_id = 1;
    trw_server_stats stats{};
    // owned by the worker thread
    std::vector<Active> active;
    std::vector<uint32_t> free_slots;
    unsigned long long tail = 0;
    std::thread worker;
    std::string fatal;

    trw_server_s(size_t pool_bytes) : pool(pool_bytes) {}
};

namespace trw {
namespace {

trw_status sfail(trw_status st, const std::string &m) {
    set_error(m);
    return st;
}

// Pool layout of an admitted request with host buffers: sources copy, paths,
// lengths, status (copied to the host at completion).  A request with device
// buffers takes no pool space: its sources are read and its outputs written
// in place.
size_t request_src_bytes(const trw_request &r) {
    return (r.flags & TRW_REQ_HOST) ? align_up(sizeof(int32_t) * (size_t)r.nq) : 0;
}

size_t request_pool_bytes(const trw_request &r) {
    if (!(r.flags & TRW_REQ_HOST)) return 0;
    const uint64_t stride = ((uint64_t)r.params.max_len + 1 + 7) / 8 * 8;
    return request_src_bytes(r) + align_up(sizeof(int32_t) * stride * r.nq) + align_up(sizeof(uint32_t) * (size_t)r.nq) +
           align_up((size_t)r.nq);
}

trw_status check_request(const trw_server_s *s, const trw_request *r) {
    if (!r) return sfail(TRW_E_INVALID, "request is NULL");
    const trw_walk_params &p = r->params;
    const bool static_walk = p.algo == TRW_A_DEEPWALK || p.algo == TRW_A_PPR;
    if (!((static_walk && (p.sampler == TRW_S_NAIVE || p.sampler == TRW_S_ALIAS)) ||
          (p.algo == TRW_A_NODE2VEC && p.sampler == TRW_S_OREJ)))
        return sfail(TRW_E_UNSUPPORTED, "served walks: DeepWalk/PPR with NAIVE or ALIAS, Node2Vec with OREJ");
    if (p.sampler == TRW_S_ALIAS && !s->t.alias) return sfail(TRW_E_INVALID, "server was created without an ALIAS table");
    if (p.max_len == 0 || p.max_len > 65535) return sfail(TRW_E_INVALID, "max_len must be in 1..65535");
    if (p.algo == TRW_A_NODE2VEC)
        for (int i = 0; i < 3; ++i)
            if (p.n2v_thr_q16[i] == 0 || p.n2v_thr_q16[i] > 65536)
                return sfail(TRW_E_INVALID, "Node2Vec thresholds must be in 1..65536");
    if (r->nq == 0) return sfail(TRW_E_INVALID, "nq must be >= 1");
    if (!r->sources || !r->paths || !r->lengths || !r->status)
        return sfail(TRW_E_INVALID, "sources / paths / lengths / status is NULL");
    if (r->path_stride < (uint64_t)p.max_len + 1) return sfail(TRW_E_INVALID, "path_stride < max_len + 1");
    if ((uint64_t)r->nq / kChunkQueries + 1 > s->ring / 2) return sfail(TRW_E_INVALID, "request has too many queries");
    return TRW_OK;
}

void server_loop(trw_server_s *s);

}  // namespace
}  // namespace trw

extern "C" {

trw_status trw_server_arena_bytes(const trw_server_cfg *cfg, size_t pool_bytes, size_t *bytes) {
    if (!cfg || !bytes) return sfail(TRW_E_INVALID, "cfg / bytes is NULL");
    const DeviceInfo di = device_info();
    const uint32_t slots = cfg->max_slots ? cfg->max_slots : (uint32_t)di.num_cus * 2048;
    const uint32_t reqs = cfg->max_requests ? cfg->max_requests : 1024;
    if (slots % kServeBlock) return sfail(TRW_E_INVALID, "max_slots must be a multiple of 256");
    const uint32_t ring = cfg->ring_chunks ? cfg->ring_chunks : (1u << 20);
    if (ring < 16 || ring > (1u << 24)) return sfail(TRW_E_INVALID, "ring_chunks must be in 16..2^24");
    *bytes = layout(slots, reqs, ring).fixed + align_up(pool_bytes);
    return TRW_OK;
}

trw_status trw_server_create(trw_graph g, trw_table alias, trw_table adjacency, const trw_server_cfg *cfg,
                             void *d_arena, size_t arena_bytes, trw_server *out);
trw_status trw_server_destroy(trw_server s);

}  // extern "C"

extern "C" trw_status trw_server_create(trw_graph g, trw_table alias, trw_table adjacency, const trw_server_cfg *cfg,
                                        void *d_arena, size_t arena_bytes, trw_server *out) {
    if (!g || !cfg || !out) return sfail(TRW_E_INVALID, "graph / cfg / out is NULL");
    const DeviceInfo di = device_info();
    const uint32_t slots = cfg->max_slots ? cfg->max_slots : (uint32_t)di.num_cus * 2048;
    const uint32_t reqs = cfg->max_requests ? cfg->max_requests : 1024;
    const uint32_t steps = cfg->steps_per_tick ? cfg->steps_per_tick : 16;
    if (slots % kServeBlock || slots > (1u << 24)) return sfail(TRW_E_INVALID, "max_slots must be a multiple of 256, <= 2^24");
    if (reqs > 65536) return sfail(TRW_E_INVALID, "max_requests must be <= 65536");
    const uint32_t ring = cfg->ring_chunks ? cfg->ring_chunks : (1u << 20);
    if (ring < 16 || ring > (1u << 24)) return sfail(TRW_E_INVALID, "ring_chunks must be in 16..2^24");
    const Layout lay = layout(slots, reqs, ring);
    if (!d_arena || (reinterpret_cast<uintptr_t>(d_arena) & 255)) return sfail(TRW_E_INVALID, "arena NULL or not 256-byte aligned");
    if (arena_bytes < lay.fixed + kA) return sfail(TRW_E_INVALID, "arena smaller than the fixed server state");
    TableDev t{nullptr, nullptr, nullptr, nullptr, 0, nullptr};
    const void *buf = nullptr;
    trw_graph tg = nullptr;
    if (alias) {
        if (!table_view(alias, TRW_S_ALIAS, &buf, &tg) || tg != g)
            return sfail(TRW_E_INVALID, "alias is not an ALIAS table of this graph");
        t.alias = static_cast<const uint4 *>(buf);
    }
    if (adjacency) {
        if (table_view(adjacency, kEdgeIndexKind, &buf, &tg) && tg == g) {
            t.eset = reinterpret_cast<const unsigned long long *>(static_cast<const char *>(buf) +
                                                                  edge_index_records_bytes(graph_dev(g).m));
            t.eset_mask = eset_slots(graph_dev(g).m) - 1;
        } else if (!table_view(adjacency, kAdjacencyKind, &buf, &tg) || tg != g) {
            return sfail(TRW_E_INVALID, "adjacency is not an adjacency or edge index of this graph");
        }
        t.adj = static_cast<const uint4 *>(buf);
    }
    auto *s = new (std::nothrow) trw_server_s(arena_bytes - lay.fixed);
    if (!s) return sfail(TRW_E_INVALID, "out of host memory");
    s->g = graph_dev(g);
    s->t = t;
    s->slots = slots; s->max_reqs = reqs; s->ring = ring; s->steps = steps;
    s->use_graph = cfg->use_hipgraph != 0;
    s->pipelined = cfg->serial_ticks == 0;
    s->device = di.device;
    s->arena = static_cast<char *>(d_arena);
    s->lay = lay;
    char *a = s->arena;
    s->dev.reqs = reinterpret_cast<ReqDesc *>(a + lay.reqs);
    s->dev.ring = reinterpret_cast<const Chunk *>(a + lay.ring);
    s->dev.ring_size = ring;
    auto *ctr = reinterpret_cast<unsigned long long *>(a + lay.counters);
    s->dev.head = ctr;
    s->dev.tail = ctr + 1;
    s->dev.done = reinterpret_cast<uint32_t *>(a + lay.done);
    s->dev.moves = reinterpret_cast<unsigned long long *>(a + lay.done + lay.done_bytes - sizeof(unsigned long long));
    s->dev.slots = reinterpret_cast<SlotState *>(a + lay.slots);
    s->dev.waves = reinterpret_cast<WaveState *>(a + lay.waves);

    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->deliver_stream, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipEventCreate(&s->tick_done[i]);
        if (e == hipSuccess) e = hipEventCreate(&s->tick_start[i]);
        if (e == hipSuccess) e = hipEventCreate(&s->tick_end[i]);
    }
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_desc, sizeof(ReqDesc) * reqs, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_ring, sizeof(Chunk) * ring, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_tail, 2 * sizeof(unsigned long long), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_done, 2 * lay.done_bytes, hipHostMallocDefault);
    if (e == hipSuccess) {
        std::memset(s->h_desc, 0, sizeof(ReqDesc) * reqs);
        std::memset(s->h_done, 0, 2 * lay.done_bytes);
        s->slot_done.assign(reqs, 0u);
    }
    if (e == hipSuccess) {
        // zero the counters, descriptors and waves; mark every slot free (0xFF bytes)
        auto fill = [&](size_t off, size_t bytes, uint32_t v) {
            hipLaunchKernelGGL(k_fill_bytes, dim3(1024), dim3(256), 0, s->stream,
                               reinterpret_cast<uint32_t *>(a + off), bytes / 4, v);
        };
        fill(lay.reqs, lay.slots - lay.reqs, 0u);
        fill(lay.slots, lay.waves - lay.slots, 0xFFFFFFFFu);
        fill(lay.waves, lay.pool - lay.waves, 0u);
        e = hipGetLastError();
    }
    if (e == hipSuccess && s->use_graph) {
        e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = launch_serve_tick(s->g, s->t, s->dev, s->steps, s->slots / kServeBlock, s->stream);
            e = hipStreamEndCapture(s->stream, &s->graph);
            if (e == hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&s->graph_exec, s->graph, nullptr, nullptr, 0);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        std::string msg = std::string("server setup: ") + hipGetErrorString(e);
        trw_server_destroy(s);
        return sfail(TRW_E_DEVICE, msg);
    }
    for (uint32_t i = 0; i < reqs; ++i) s->free_slots.push_back(reqs - 1 - i);
    s->worker = std::thread([s] { server_loop(s); });
    *out = s;
    return TRW_OK;
}

extern "C" trw_status trw_server_request_bytes(trw_server s, const trw_request *r, size_t *bytes) {
    if (!s || !bytes) return sfail(TRW_E_INVALID, "server / bytes is NULL");
    trw_status st = check_request(s, r);
    if (st != TRW_OK) return st;
    *bytes = request_pool_bytes(*r);
    return TRW_OK;
}

extern "C" trw_status trw_server_submit(trw_server s, const trw_request *r, uint64_t *request_id) {
    if (!s || !request_id) return sfail(TRW_E_INVALID, "server / request_id is NULL");
    trw_status st = check_request(s, r);
    if (st != TRW_OK) return st;
    const size_t bytes = request_pool_bytes(*r);
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->fatal.empty()) return sfail(TRW_E_DEVICE, s->fatal);
    if (s->stopping) return sfail(TRW_E_CANCELLED, "server is shutting down");
    if (bytes > s->pool.size()) {
        s->stats.rejected++;
        return sfail(TRW_E_NOMEM_BUDGET, "request needs " + std::to_string(bytes) + " bytes, the pool has " +
                                             std::to_string(s->pool.size()));
    }
    const uint64_t id = s->next_id++;
    s->waiting.push_back(Pending{id, *r, now_ns(), bytes});
    s->stats.submitted++;
    *request_id = id;
    s->cv_work.notify_one();
    return TRW_OK;
}

extern "C" trw_status trw_server_cancel(trw_server s, uint64_t request_id) {
    if (!s) return sfail(TRW_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    s->cancel_requests.push_back(request_id);
    s->cv_work.notify_one();
    return TRW_OK;
}

extern "C" trw_status trw_server_poll(trw_server s, trw_completion *out, uint32_t max, uint32_t *n_out,
                                      uint32_t timeout_ms) {
    if (!s || !n_out || (!out && max)) return sfail(TRW_E_INVALID, "server / out / n_out is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->completed.empty() && timeout_ms)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                            [s] { return !s->completed.empty() || !s->fatal.empty(); });
    uint32_t n = 0;
    while (n < max && !s->completed.empty()) {
        out[n++] = s->completed.front();
        s->completed.pop_front();
    }
    *n_out = n;
    if (!s->fatal.empty() && n == 0) return sfail(TRW_E_DEVICE, s->fatal);
    if (n == 0 && timeout_ms) return sfail(TRW_E_TIMEOUT, "no request completed in time");
    return TRW_OK;
}

extern "C" trw_status trw_server_stats_get(trw_server s, trw_server_stats *out) {
    if (!s || !out) return sfail(TRW_E_INVALID, "server / out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->waiting = (uint32_t)s->waiting.size();
    out->pool_bytes = s->pool.size();
    return TRW_OK;
}

extern "C" trw_status trw_server_destroy(trw_server s) {
    if (!s) return TRW_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->deliver_stream) (void)hipStreamSynchronize(s->deliver_stream);
    for (int i = 0; i < 2; ++i) {
        if (s->tick_done[i]) (void)hipEventDestroy(s->tick_done[i]);
        if (s->tick_start[i]) (void)hipEventDestroy(s->tick_start[i]);
        if (s->tick_end[i]) (void)hipEventDestroy(s->tick_end[i]);
    }
    for (auto &b : s->batches)
        if (b.done) (void)hipEventDestroy(b.done);
    for (auto ev : s->spare_events) (void)hipEventDestroy(ev);
    if (s->h_desc) (void)hipHostFree(s->h_desc);
    if (s->h_ring) (void)hipHostFree(s->h_ring);
    if (s->h_tail) (void)hipHostFree(s->h_tail);
    if (s->h_done) (void)hipHostFree(s->h_done);
    if (s->deliver_stream) (void)hipStreamDestroy(s->deliver_stream);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return TRW_OK;
}

namespace trw {
namespace {

// The requests of delivered batch `seq` complete: their pool ranges and
// request slots are freed, and their completions are handed over under one
// lock with one wake-up.
void complete_batch(trw_server_s *s, uint64_t seq) {
    std::vector<trw_completion> out;
    const uint64_t t = now_ns();
    for (const Active &a : s->active) {
        if (!a.finishing || a.batch_seq != seq) continue;
        trw_completion c{};
        c.request_id = a.id;
        c.status = a.cancelled ? TRW_E_CANCELLED : TRW_OK;
        c.nq = a.req.nq;
        c.user = a.req.user;
        c.t_submit_ns = a.t_submit;
        c.t_admit_ns = a.t_admit;
        c.t_done_ns = t;
        if (a.pool_bytes) s->pool.release(a.pool_off, a.pool_bytes);
        s->slot_done[a.slot] = a.done_base + a.req.nq;    // every query of a request counts once
        s->free_slots.push_back(a.slot);
        out.push_back(c);
    }
    s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                   [seq](const Active &a) { return a.finishing && a.batch_seq == seq; }),
                    s->active.end());
    std::lock_guard<std::mutex> lk(s->mu);
    for (const trw_completion &c : out) {
        s->completed.push_back(c);
        if (c.status == TRW_OK) s->stats.completed++; else s->stats.cancelled++;
    }
    s->stats.active = (uint32_t)s->active.size();
    s->cv_done.notify_all();
}

void desc_touch(trw_server_s *s, uint32_t i) {
    if (s->desc_hi == s->desc_lo) {
        s->desc_lo = i;
        s->desc_hi = i + 1;
    } else {
        s->desc_lo = std::min(s->desc_lo, i);
        s->desc_hi = std::max(s->desc_hi, i + 1);
    }
}

// Admit waiting requests while a slot, pool space and ring entries are free
// (first come, first served), then publish the descriptor table, the new
// chunks and the tail.  The chunks admitted together are published grouped
// by walk kind (algorithm and sampler), in admission order within a kind:
// waves take chunks in ring order, so a wave's lanes then mostly run one kind
// of move, and a wave does not step at the pace of its slowest kind.
//
// Ring entries: the device may still read a published chunk only while its
// request has queries not yet counted done (a query is counted once its walk
// ends or it is cancelled, both after its chunk was read).  So every entry the
// device may still read lies in [oldest, tail), where `oldest` is the first
// chunk of the oldest admitted request not yet known to be finished.  New
// chunks go to [tail, tail + c); they overwrite none of those entries as long
// as tail + c - oldest <= ring.
hipError_t admit(trw_server_s *s, std::deque<Pending> &incoming, int half) {
    hipError_t e = hipSuccess;
    const unsigned long long tail0 = s->tail;
    unsigned long long oldest = s->tail;
    for (const Active &a : s->active)
        if (!a.finishing) oldest = std::min(oldest, a.first_chunk);
    const size_t first_new = s->active.size();
    unsigned long long new_chunks = 0;
    while (!incoming.empty() && !s->free_slots.empty()) {
        Pending &p = incoming.front();
        const unsigned long long chunks = (p.req.nq + kChunkQueries - 1) / kChunkQueries;
        if (tail0 + new_chunks + chunks - oldest > s->ring) break;
        size_t off = 0;
        if (p.bytes && !s->pool.alloc(p.bytes, &off)) break;
        const uint32_t slot = s->free_slots.back();
        s->free_slots.pop_back();
        const trw_request &r = p.req;
        const bool in_place = !(r.flags & TRW_REQ_HOST);
        const uint64_t stride = in_place ? r.path_stride : ((uint64_t)r.params.max_len + 1 + 7) / 8 * 8;
        char *base = s->arena + s->lay.pool + off;
        const size_t src_bytes = request_src_bytes(r);
        const int32_t *src = static_cast<const int32_t *>(r.sources);
        if (r.flags & TRW_REQ_HOST) {
            e = hipMemcpyAsync(base, r.sources, sizeof(int32_t) * r.nq, hipMemcpyHostToDevice, s->stream);
            if (e != hipSuccess) return e;
            src = reinterpret_cast<const int32_t *>(base);
        }
        int32_t *paths = r.paths;
        uint32_t *lengths = r.lengths;
        uint8_t *status = r.status;
        if (!in_place) {                       // staged in the pool, copied to the host at completion
            paths = reinterpret_cast<int32_t *>(base + src_bytes);
            lengths = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(paths) +
                                                   align_up(sizeof(int32_t) * stride * r.nq));
            status = reinterpret_cast<uint8_t *>(reinterpret_cast<char *>(lengths) +
                                                 align_up(sizeof(uint32_t) * (size_t)r.nq));
        }
        ReqDesc &d = s->h_desc[slot];
        std::memset(&d, 0, sizeof(d));
        d.algo = r.params.algo;
        d.sampler = r.params.sampler;
        d.max_len = r.params.max_len;
        d.stop_q32 = r.params.algo == TRW_A_PPR ? r.params.stop_q32 : 0;
        for (int i = 0; i < 3; ++i) d.thr[i] = r.params.n2v_thr_q16[i];
        d.seed = r.params.seed;
        d.qid_base = r.qid_base;
        d.sources = src;
        d.paths = paths;
        d.lengths = lengths;
        d.status = status;
        d.stride = stride;
        d.nq = r.nq;
        desc_touch(s, slot);
        new_chunks += chunks;
        Active a;
        a.id = p.id; a.req = r; a.t_submit = p.t_submit; a.t_admit = now_ns();
        a.pool_off = off; a.pool_bytes = p.bytes; a.slot = slot; a.stride = stride;
        a.first_chunk = 0;                  // set below, when the chunks are placed
        a.done_base = s->slot_done[slot];   // the counter is not reset between requests
        a.out_off = src_bytes;
        s->active.push_back(a);
        incoming.pop_front();
    }
    // Place the new requests' chunks in [tail0, tail0 + new_chunks), kind by kind.
    std::vector<size_t> order(s->active.size() - first_new);
    for (size_t i = 0; i < order.size(); ++i) order[i] = first_new + i;
    auto kind = [&](size_t i) { return s->active[i].req.params.algo * 16u + s->active[i].req.params.sampler; };
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return kind(x) < kind(y); });
    for (size_t i : order) {
        Active &a = s->active[i];
        a.first_chunk = s->tail;
        for (uint32_t b = 0; b < a.req.nq; b += kChunkQueries) {
            Chunk &c = s->h_ring[s->tail % s->ring];
            c.req = a.slot; c.begin = b; c.end = std::min<uint32_t>(a.req.nq, b + kChunkQueries); c.pad = 0;
            s->tail++;
        }
    }
    if (s->desc_hi > s->desc_lo) {            // the changed range of the descriptor table only
        e = hipMemcpyAsync(s->dev.reqs + s->desc_lo, s->h_desc + s->desc_lo, sizeof(ReqDesc) * (s->desc_hi - s->desc_lo),
                           hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return e;
        s->desc_lo = s->desc_hi = 0;
    }
    if (s->tail == tail0) return hipSuccess;
    // copy the new ring entries (they may wrap around), then publish the tail
    for (unsigned long long i = tail0; i < s->tail;) {
        const unsigned long long pos = i % s->ring;
        const unsigned long long n = std::min<unsigned long long>(s->tail - i, s->ring - pos);
        e = hipMemcpyAsync(const_cast<Chunk *>(s->dev.ring) + pos, s->h_ring + pos, sizeof(Chunk) * n,
                           hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return e;
        i += n;
    }
    // this half is not read by a pending copy: that copy preceded tick i-2, which has ended
    s->h_tail[half] = s->tail;
    return hipMemcpyAsync(const_cast<unsigned long long *>(s->dev.tail), &s->h_tail[half], sizeof(unsigned long long),
                          hipMemcpyHostToDevice, s->stream);
}

// Outputs of a finished request: 2D copy of the path rows, lengths, status.
void output_jobs(const trw_server_s *s, const Active &a, CopyJob *jobs) {
    const trw_request &r = a.req;
    const char *base = s->arena + s->lay.pool + a.pool_off + a.out_off;
    const char *paths = base;
    const char *lengths = paths + align_up(sizeof(int32_t) * a.stride * r.nq);
    const char *status = lengths + align_up(sizeof(uint32_t) * (size_t)r.nq);
    jobs[0] = CopyJob{paths, reinterpret_cast<char *>(r.paths), sizeof(int32_t) * a.stride,
                      sizeof(int32_t) * r.path_stride, sizeof(int32_t) * ((size_t)r.params.max_len + 1), r.nq};
    jobs[1] = CopyJob{lengths, reinterpret_cast<char *>(r.lengths), 0, 0, sizeof(uint32_t) * (size_t)r.nq, 1};
    jobs[2] = CopyJob{status, reinterpret_cast<char *>(r.status), 0, 0, (size_t)r.nq, 1};
}

void server_loop(trw_server_s *s) {
    (void)hipSetDevice(s->device);
    std::deque<Pending> incoming, empty;
    int cur = 0;                  // half of the staging buffers the next tick uses
    bool prev_launched = false;   // a tick was enqueued in the previous pass and not yet read
    for (;;) {
        std::vector<uint64_t> cancels;
        bool stopping;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->active.empty() && s->waiting.empty() && incoming.empty() && s->cancel_requests.empty() &&
                !s->stopping && !prev_launched && s->batches.empty())
                s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            while (!s->waiting.empty()) {
                incoming.push_back(s->waiting.front());
                s->waiting.pop_front();
            }
            cancels.swap(s->cancel_requests);
            stopping = s->stopping;
        }
        if (stopping) {
            for (auto &p : incoming) cancels.push_back(p.id);
            for (auto &a : s->active) cancels.push_back(a.id);
        }
        // cancellations: not yet admitted -> done at once; running -> flag the descriptor
        for (uint64_t id : cancels) {
            for (auto it = incoming.begin(); it != incoming.end(); ++it) {
                if (it->id == id) {
                    trw_completion c{};
                    c.request_id = id; c.status = TRW_E_CANCELLED; c.nq = it->req.nq; c.user = it->req.user;
                    c.t_submit_ns = it->t_submit; c.t_done_ns = now_ns();
                    incoming.erase(it);
                    std::lock_guard<std::mutex> lk(s->mu);
                    s->completed.push_back(c);
                    s->stats.cancelled++;
                    s->cv_done.notify_all();
                    break;
                }
            }
            for (auto &a : s->active) {
                if (a.id == id && !a.cancelled && !a.finishing) {
                    a.cancelled = true;
                    s->h_desc[a.slot].cancelled = 1;
                    desc_touch(s, a.slot);
                }
            }
        }
        hipError_t e = admit(s, stopping ? empty : incoming, cur);
        // Enqueue tick `cur` (it runs after the copies admit() queued), then
        // take the previous tick's counters while this one runs.
        bool launched = false;
        if (e == hipSuccess) {
            bool running = false;
            for (auto &a : s->active) running |= !a.finishing;
            if (running) {
                uint32_t *done_half = s->h_done + cur * (s->lay.done_bytes / sizeof(uint32_t));
                e = hipEventRecord(s->tick_start[cur], s->stream);
                if (e == hipSuccess)
                    e = s->use_graph ? hipGraphLaunch(s->graph_exec, s->stream)
                                     : launch_serve_tick(s->g, s->t, s->dev, s->steps, s->slots / kServeBlock, s->stream);
                if (e == hipSuccess) e = hipEventRecord(s->tick_end[cur], s->stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(done_half, s->dev.done, s->lay.done_bytes, hipMemcpyDeviceToHost, s->stream);
                if (e == hipSuccess) e = hipEventRecord(s->tick_done[cur], s->stream);
                launched = e == hipSuccess;
            }
        }
        // The tick whose counters are read now: the previous one when pipelined
        // (the current one is queued behind it), else the one just queued.
        const bool read_tick = s->pipelined ? prev_launched : launched;
        hipStream_t out_stream = s->pipelined ? s->deliver_stream : s->stream;
        if (e == hipSuccess && read_tick) {
            const int prev = s->pipelined ? (cur ^ 1) : cur;
            e = hipEventSynchronize(s->tick_done[prev]);
            const uint32_t *done_prev = s->h_done + prev * (s->lay.done_bytes / sizeof(uint32_t));
            if (e == hipSuccess) {
                unsigned long long mv;
                std::memcpy(&mv, reinterpret_cast<const char *>(done_prev) + s->lay.done_bytes - sizeof(mv), sizeof(mv));
                float ms = 0;
                (void)hipEventElapsedTime(&ms, s->tick_start[prev], s->tick_end[prev]);
                std::lock_guard<std::mutex> lk(s->mu);
                s->stats.ticks++;
                s->stats.moves = mv;
                s->stats.tick_device_ns += (uint64_t)(ms * 1e6);
            }
            // Requests that finished by that tick.  Device outputs were written in
            // place by the ticks; host outputs are copied out of the pool, pipelined:
            // on the delivery stream while the next tick runs (it touches none of
            // them); serial: on the tick stream, ahead of the next tick.
            Batch batch;
            batch.seq = s->n_batches;
            bool any_copy = false;
            for (size_t i = 0; i < s->active.size() && e == hipSuccess; ++i) {
                Active &a = s->active[i];
                if (a.finishing || done_prev[a.slot] - a.done_base < a.req.nq) continue;
                a.finishing = true;
                a.batch_seq = batch.seq;
                batch.ids.push_back(a.id);
                if (a.cancelled || !(a.req.flags & TRW_REQ_HOST)) continue;
                CopyJob jobs[3];
                output_jobs(s, a, jobs);
                e = hipMemcpy2DAsync(jobs[0].dst, jobs[0].dst_pitch, jobs[0].src, jobs[0].src_pitch, jobs[0].width,
                                     jobs[0].rows, hipMemcpyDeviceToHost, out_stream);
                for (int k = 1; k < 3 && e == hipSuccess; ++k)
                    e = hipMemcpyAsync(jobs[k].dst, jobs[k].src, jobs[k].width, hipMemcpyDeviceToHost, out_stream);
                any_copy = true;
            }
            if (e == hipSuccess && !batch.ids.empty()) {
                if (any_copy) {
                    if (!s->spare_events.empty()) {
                        batch.done = s->spare_events.back();
                        s->spare_events.pop_back();
                    } else {
                        e = hipEventCreateWithFlags(&batch.done, hipEventDisableTiming);
                    }
                    if (e == hipSuccess) e = hipEventRecord(batch.done, out_stream);
                }
                s->n_batches++;
                s->batches.push_back(std::move(batch));
            }
        }
        // Complete the batches whose copies have ended, in order.
        while (e == hipSuccess && !s->batches.empty()) {
            Batch &b = s->batches.front();
            if (b.done) {
                hipError_t q = hipEventQuery(b.done);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) { e = q; break; }
                s->spare_events.push_back(b.done);
            }
            complete_batch(s, b.seq);
            s->batches.pop_front();
        }
        prev_launched = s->pipelined && launched;
        cur ^= 1;
        if (e != hipSuccess) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->fatal = std::string("server device error: ") + hipGetErrorString(e);
            s->cv_done.notify_all();
            return;
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stats.active = (uint32_t)s->active.size();
            s->stats.pool_bytes_used = s->pool.used();
        }
        if (stopping && s->active.empty() && incoming.empty() && !prev_launched && s->batches.empty()) return;
        bool copies_only = !s->active.empty() && !prev_launched;
        for (auto &a : s->active) copies_only &= a.finishing;
        if (copies_only) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace
}  // namespace trw
