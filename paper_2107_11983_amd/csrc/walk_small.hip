// Walks on graphs small enough to live in one workgroup's LDS.
//
// A DeepWalk or PPR move with uniform sampling (NAIVE) reads the current
// vertex's row range and one destination of that row.  When the CSR arrays
// fit in the LDS a gfx950 workgroup may allocate (160 KiB: row offsets as
// int32, destinations as uint16, so 4(n+1) + 2m bytes and at most 65536
// vertices), every workgroup copies the graph into LDS once and its moves
// read LDS from then on instead of L2 or HBM.  The walk is otherwise the
// persistent walk: the same random blocks (Philox counter (k, 0, query id)),
// the same index map, the same termination tests and the same outputs, so the
// results are identical; lanes refill from the same device queue.
#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "trw_device.hpp"
#include "trw_internal.hpp"

namespace trw {
namespace {

constexpr uint32_t kSmallIdle = 0xFFFFFFFFu;
constexpr size_t kSmallMaxVertices = 65536;      // destinations stored as uint16

size_t round16(size_t b) { return (b + 15) / 16 * 16; }

size_t small_rp_bytes(const GraphDev &g) { return round16(sizeof(int32_t) * ((size_t)g.n + 1)); }

size_t small_lds_bytes(const GraphDev &g) { return small_rp_bytes(g) + round16(sizeof(uint16_t) * (size_t)g.m); }

// The graph into LDS.  The copy is latency-bound (a workgroup moves up to
// 160 KiB once, before its first move), so each thread keeps kFillBatch
// 16-byte loads in flight; arrays that do not start on 16 bytes are copied
// entry by entry.
constexpr int kFillBatch = 16;

__device__ __forceinline__ void put16(uint2 *dst, uint32_t i, const int4 &v) {
    dst[i] = make_uint2(((uint32_t)v.x & 0xFFFFu) | ((uint32_t)v.y << 16),
                        ((uint32_t)v.z & 0xFFFFu) | ((uint32_t)v.w << 16));
}

__device__ void fill_lds(const GraphDev &g, int32_t *rp, uint16_t *c16) {
    const uint32_t n1 = (uint32_t)g.n + 1, m = (uint32_t)g.m, t = threadIdx.x, T = blockDim.x;
    const bool vec = ((reinterpret_cast<uintptr_t>(g.row_ptr) | reinterpret_cast<uintptr_t>(g.col)) & 15) == 0;
    const uint32_t r4 = vec ? n1 / 4 : 0, c4 = vec ? m / 4 : 0;
    const int4 *rs = reinterpret_cast<const int4 *>(g.row_ptr);
    const int4 *cs = reinterpret_cast<const int4 *>(g.col);
    int4 *rd = reinterpret_cast<int4 *>(rp);
    uint2 *cd = reinterpret_cast<uint2 *>(c16);
    uint32_t i = t;
    for (; i + (kFillBatch - 1) * T < r4; i += kFillBatch * T) {
        int4 v[kFillBatch];
#pragma unroll
        for (int j = 0; j < kFillBatch; ++j) v[j] = rs[i + j * T];
#pragma unroll
        for (int j = 0; j < kFillBatch; ++j) rd[i + j * T] = v[j];
    }
    for (; i < r4; i += T) rd[i] = rs[i];
    i = t;
    for (; i + (kFillBatch - 1) * T < c4; i += kFillBatch * T) {
        int4 v[kFillBatch];
#pragma unroll
        for (int j = 0; j < kFillBatch; ++j) v[j] = cs[i + j * T];
#pragma unroll
        for (int j = 0; j < kFillBatch; ++j) put16(cd, i + j * T, v[j]);
    }
    for (; i < c4; i += T) put16(cd, i, cs[i]);
    for (i = 4 * r4 + t; i < n1; i += T) rp[i] = g.row_ptr[i];
    for (i = 4 * c4 + t; i < m; i += T) c16[i] = (uint16_t)g.col[i];
}

__global__ void k_small_zero_head(unsigned long long *head) {
    if (threadIdx.x == 0) *head = 0;
}

template <uint32_t ALGO>
__global__ void __launch_bounds__(1024)
k_walk_small(GraphDev g, WalkDev a, unsigned long long *__restrict__ queue_head, uint32_t rp_bytes) {
    extern __shared__ __align__(16) unsigned char small_lds[];
    int32_t *rp = reinterpret_cast<int32_t *>(small_lds);
    uint16_t *c16 = reinterpret_cast<uint16_t *>(small_lds + rp_bytes);

    fill_lds(g, rp, c16);
    __syncthreads();

    const uint32_t lane = lane_id();
    uint32_t qi = kSmallIdle, k = 0;
    int32_t cur = 0;
    PathBuf path;
    bool exhausted = false;       // wave-uniform: the queue has nothing left for this wave
    while (true) {
        // Idle lanes take the next query ids: one atomic per wave.
        const uint64_t want = __ballot(qi == kSmallIdle && !exhausted);
        if (want != 0) {
            const uint32_t cnt = (uint32_t)__popcll(want);
            const int leader = (int)__builtin_ctzll(want);
            unsigned long long base = 0;
            if (lane == (uint32_t)leader) base = atomicAdd(queue_head, (unsigned long long)cnt);
            base = __shfl(base, leader);
            if (base + cnt >= a.nq) exhausted = true;
            if ((want >> lane) & 1ull) {
                const unsigned long long q = base + rank_below(want);
                if (q < a.nq) {
                    const int32_t s = a.sources[q];
                    if (s < 0 || s >= g.n) {
                        a.lengths[q] = 0;
                        a.status[q] = ST_BAD_SOURCE;
                    } else {
                        qi = (uint32_t)q;
                        k = 0;
                        cur = s;
                        path.start(a.paths + q * a.stride);
                        path.push(s);
                    }
                }
            }
        }
        const bool act = qi != kSmallIdle;
        if (__ballot(act) == 0) {
            if (exhausted) break;
            continue;
        }
        if (act) {
            const Rand4 r = philox(k, 0u, a.qid_base + qi, a.seed);
            const int32_t off = rp[cur];
            const uint32_t d = (uint32_t)(rp[cur + 1] - off);
            uint8_t st = 0;
            if (d == 0) {
                st = ST_DEAD_END;
            } else {
                const int32_t nxt = (int32_t)c16[off + scale32(r.r0, d)];
                path.push(nxt);
                cur = nxt;
                ++k;
                if (ALGO == ALG_PPR && r.r2 < a.stop_q32) st = ST_STOPPED;
                else if (k == a.max_len) st = ST_LENGTH;
            }
            if (st) {
                path.finish(a.paths + ((uint64_t)qi + 1) * a.stride);
                a.lengths[qi] = k;
                a.status[qi] = st;
                qi = kSmallIdle;
            }
        }
    }
}

}  // namespace

bool small_graph_fits(const GraphDev &g, const DeviceInfo &di) {
    return (size_t)g.n <= kSmallMaxVertices && small_lds_bytes(g) <= (size_t)di.lds_per_block;
}

hipError_t launch_walk_small(const GraphDev &g, const WalkDev &w, uint32_t algo, const DeviceInfo &di, void *ws,
                             hipStream_t s) {
    auto *head = reinterpret_cast<unsigned long long *>(ws);
    hipLaunchKernelGGL(k_small_zero_head, dim3(1), dim3(64), 0, s, head);
    // One workgroup per CU (the graph takes most of the LDS).  Few queries:
    // 256 lanes per workgroup, spread over more CUs; many: 1024, so that
    // each SIMD has four waves to switch between.
    const uint32_t threads = (uint64_t)w.nq <= 256ull * di.num_cus ? 256 : 1024;
    const uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>(((uint64_t)w.nq + threads - 1) / threads,
                                                                     (uint64_t)di.num_cus));
    const size_t lds = small_lds_bytes(g);
    const uint32_t rpb = (uint32_t)small_rp_bytes(g);
    const void *fn = algo == ALG_PPR ? reinterpret_cast<const void *>(&k_walk_small<ALG_PPR>)
                                     : reinterpret_cast<const void *>(&k_walk_small<ALG_DEEPWALK>);
    // Dynamic LDS above 64 KiB: declared to the runtime once per kernel and
    // device, for the most any graph can ask; a launch reports any refusal itself.
    {
        static std::mutex mu;
        static std::vector<std::pair<int, const void *>> done;
        std::lock_guard<std::mutex> lk(mu);
        if (std::find(done.begin(), done.end(), std::make_pair(di.device, fn)) == done.end()) {
            if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, di.lds_per_block) != hipSuccess)
                (void)hipGetLastError();
            done.emplace_back(di.device, fn);
        }
    }
    if (algo == ALG_PPR)
        hipLaunchKernelGGL(k_walk_small<ALG_PPR>, dim3(blocks), dim3(threads), lds, s, g, w, head, rpb);
    else
        hipLaunchKernelGGL(k_walk_small<ALG_DEEPWALK>, dim3(blocks), dim3(threads), lds, s, g, w, head, rpb);
    return hipGetLastError();
}

}  // namespace trw
