// PPR estimate (Random Walk based Algorithms, PPR): a vertex's score for a
// source is the share of that source's queries whose walk ends there.  Two
// device steps over a walk's outputs:
//  * end counts: a thread per query reads its length, status and end vertex
//    and adds one to counts[group][end];
//  * top-k: the k highest counts, ties to the smaller id, by a radix select
//    over the unique 64-bit keys count << 32 | ~id.  Eight passes, one per
//    byte from the top, each histogram the keys that agree with the bytes
//    chosen so far and let one workgroup choose the next byte; what remains
//    is exactly the k-th largest key.  The keys at or above it (k of them)
//    are then gathered and sorted in LDS.  Everything stays on the device:
//    no host round trip between passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "trw_device.hpp"
#include "trw_internal.hpp"

namespace trw {
namespace {

constexpr uint32_t kTopkMax = 4096;
constexpr size_t kTopkStateOffset = 1024;   // after uint32 hist[256]
constexpr size_t kTopkSelOffset = 1280;     // uint64 keys[k]

struct TopkState {
    unsigned long long prefix;   // bytes of the k-th key chosen so far
    uint32_t k_left;             // its rank among the keys that agree with them
    uint32_t n_sel;              // keys gathered
};

__device__ __forceinline__ unsigned long long topk_key(uint32_t count, uint32_t v) {
    return ((unsigned long long)count << 32) | (0xFFFFFFFFu - v);
}

__global__ void __launch_bounds__(256) k_end_counts(const int32_t *__restrict__ paths, uint64_t stride,
                                                   const uint32_t *__restrict__ lengths,
                                                   const uint8_t *__restrict__ status, uint64_t nq, uint64_t group,
                                                   int64_t n, uint32_t *__restrict__ counts,
                                                   unsigned long long *__restrict__ skipped) {
    uint32_t skip = 0;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t len = lengths[q];
        bool ok = status[q] != ST_BAD_SOURCE && (uint64_t)len < stride;
        const int32_t v = ok ? paths[q * stride + len] : -1;
        ok = ok && v >= 0 && (int64_t)v < n;
        if (ok) atomicAdd(&counts[(group ? q / group : 0) * (uint64_t)n + (uint32_t)v], 1u);
        else ++skip;
    }
    if (skipped) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) skip += __shfl_xor(skip, o);
        if (lane_id() == 0 && skip) atomicAdd(skipped, (unsigned long long)skip);
    }
}

__global__ void k_topk_init(uint32_t *ws, uint32_t k) {
    ws[threadIdx.x] = 0;                    // 256 threads: the histogram
    if (threadIdx.x == 0) {
        auto *st = reinterpret_cast<TopkState *>(reinterpret_cast<char *>(ws) + kTopkStateOffset);
        st->prefix = 0;
        st->k_left = k;
        st->n_sel = 0;
    }
}

// Histogram of byte (key >> shift) & 255 over the keys whose higher bytes
// equal the prefix.  256 threads per block.
__global__ void __launch_bounds__(256) k_topk_hist(const uint32_t *__restrict__ counts, uint32_t n, uint32_t *ws,
                                                  uint32_t shift) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const auto *st = reinterpret_cast<const TopkState *>(reinterpret_cast<const char *>(ws) + kTopkStateOffset);
    const unsigned long long prefix = st->prefix;
    for (uint64_t base = (uint64_t)blockIdx.x * 256; base < n; base += (uint64_t)gridDim.x * 256) {
        const uint64_t v = base + threadIdx.x;
        bool in = false;
        uint32_t d = 0;
        if (v < n) {
            const unsigned long long key = topk_key(counts[v], (uint32_t)v);
            in = shift == 56 || ((key ^ prefix) >> (shift + 8)) == 0;
            d = (uint32_t)(key >> shift) & 255u;
        }
        // most waves see one byte value only (the top bytes of small counts):
        // then one LDS atomic for the wave
        const uint64_t act = __ballot(in);
        if (act) {
            const uint32_t d0 = __shfl(d, (int)__builtin_ctzll(act));
            if (__ballot(in && d == d0) == act) {
                if (lane_id() == (uint32_t)__builtin_ctzll(act)) atomicAdd(&h[d0], (uint32_t)__popcll(act));
            } else if (in) {
                atomicAdd(&h[d], 1u);
            }
        }
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&ws[threadIdx.x], h[threadIdx.x]);
}

// Choose the byte at `shift` of the k-th largest key from the histogram and
// clear the histogram for the next pass.  One block of 256 threads.
__global__ void __launch_bounds__(256) k_topk_select(uint32_t *ws, uint32_t shift) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = ws[threadIdx.x];
    ws[threadIdx.x] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        auto *st = reinterpret_cast<TopkState *>(reinterpret_cast<char *>(ws) + kTopkStateOffset);
        uint32_t k_left = st->k_left;
        uint32_t d = 255;
        // at least k_left keys agree with the prefix, so some byte holds the rank
        while (d > 0 && h[d] < k_left) {
            k_left -= h[d];
            --d;
        }
        st->k_left = k_left;
        st->prefix |= (unsigned long long)d << shift;
    }
}

// The keys at or above the k-th largest: exactly k of them (keys are unique).
__global__ void __launch_bounds__(256) k_topk_collect(const uint32_t *__restrict__ counts, uint32_t n, uint32_t *ws,
                                                     uint32_t k) {
    auto *st = reinterpret_cast<TopkState *>(reinterpret_cast<char *>(ws) + kTopkStateOffset);
    auto *sel = reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(ws) + kTopkSelOffset);
    const unsigned long long kth = st->prefix;
    for (uint64_t base = (uint64_t)blockIdx.x * 256; base < n; base += (uint64_t)gridDim.x * 256) {
        const uint64_t v = base + threadIdx.x;
        unsigned long long key = 0;
        bool take = false;
        if (v < n) {
            key = topk_key(counts[v], (uint32_t)v);
            take = key >= kth;
        }
        const uint32_t slot = wave_append(&st->n_sel, take);
        if (take && slot < k) sel[slot] = key;
    }
}

// Sort the k gathered keys, largest first (bitonic network in LDS), and
// split them into ids and counts.  One block of 1024 threads.
__global__ void __launch_bounds__(1024) k_topk_sort(const uint32_t *ws, uint32_t k, int32_t *__restrict__ ids,
                                                   uint32_t *__restrict__ vals) {
    __shared__ unsigned long long s[kTopkMax];
    const auto *sel = reinterpret_cast<const unsigned long long *>(reinterpret_cast<const char *>(ws) + kTopkSelOffset);
    uint32_t P = 1;
    while (P < k) P <<= 1;
    for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) s[i] = i < k ? sel[i] : 0ull;   // 0 is below every key
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
                const uint32_t j = i ^ stride;
                if (j > i) {
                    const unsigned long long a = s[i], b = s[j];
                    if ((i & size) == 0 ? a < b : a > b) {
                        s[i] = b;
                        s[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < k; i += blockDim.x) {
        const unsigned long long key = s[i];
        ids[i] = (int32_t)(0xFFFFFFFFu - (uint32_t)key);
        vals[i] = (uint32_t)(key >> 32);
    }
}

trw_status pfail(trw_status st, const std::string &m) {
    set_error(m);
    return st;
}

uint32_t grid_for(uint64_t items, uint32_t per_cu) {
    const uint64_t want = (items + 255) / 256;
    const uint64_t cap = (uint64_t)device_info().num_cus * per_cu;
    return (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
}

}  // namespace
}  // namespace trw

using namespace trw;

extern "C" {

trw_status trw_ppr_end_counts(trw_graph g, const int32_t *d_paths, uint64_t path_stride, const uint32_t *d_lengths,
                              const uint8_t *d_status, uint64_t nq, uint64_t group, uint32_t *d_counts,
                              uint64_t counts_len, unsigned long long *d_skipped, trw_stream_t stream) {
    if (!g) return pfail(TRW_E_INVALID, "graph is NULL");
    if (nq >= (uint64_t(1) << 32)) return pfail(TRW_E_INVALID, "nq must be < 2^32");
    if (path_stride == 0) return pfail(TRW_E_INVALID, "path_stride must be >= 1");
    const int64_t n = graph_dev(g).n;
    const uint64_t groups = group ? (nq + group - 1) / group : 1;
    if (counts_len < std::max<uint64_t>(groups, 1) * (uint64_t)n)
        return pfail(TRW_E_INVALID, "counts holds fewer than groups * n entries");
    if (nq == 0) return TRW_OK;
    if (!d_paths || !d_lengths || !d_status || !d_counts)
        return pfail(TRW_E_INVALID, "paths / lengths / status / counts is NULL");
    auto s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_end_counts, dim3(grid_for(nq, 8)), dim3(256), 0, s, d_paths, path_stride, d_lengths,
                       d_status, nq, group, n, d_counts, d_skipped);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return pfail(TRW_E_DEVICE, std::string("end counts launch: ") + hipGetErrorString(e));
    return TRW_OK;
}

trw_status trw_topk_workspace_bytes(uint64_t n, uint32_t k, size_t *bytes) {
    if (!bytes) return pfail(TRW_E_INVALID, "bytes is NULL");
    if (k > kTopkMax) return pfail(TRW_E_INVALID, "k must be <= 4096");
    if (k > n) return pfail(TRW_E_INVALID, "k must be <= n");
    *bytes = kTopkSelOffset + sizeof(unsigned long long) * (size_t)k;
    return TRW_OK;
}

trw_status trw_topk(const uint32_t *d_counts, uint64_t n, uint32_t k, int32_t *d_ids, uint32_t *d_vals,
                    void *d_ws, size_t ws_bytes, trw_stream_t stream) {
    if (n >= (uint64_t(1) << 31)) return pfail(TRW_E_INVALID, "n must be < 2^31");
    size_t need = 0;
    trw_status st = trw_topk_workspace_bytes(n, k, &need);
    if (st != TRW_OK) return st;
    if (k == 0) return TRW_OK;
    if (!d_counts || !d_ids || !d_vals) return pfail(TRW_E_INVALID, "counts / ids / vals is NULL");
    if (!d_ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_ws) & 255))
        return pfail(TRW_E_INVALID, "workspace NULL, too small or not 256-byte aligned");
    auto s = static_cast<hipStream_t>(stream);
    auto *ws = static_cast<uint32_t *>(d_ws);
    const uint32_t blocks = grid_for(n, 4);
    hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, s, ws, k);
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_topk_hist, dim3(blocks), dim3(256), 0, s, d_counts, (uint32_t)n, ws, (uint32_t)shift);
        hipLaunchKernelGGL(k_topk_select, dim3(1), dim3(256), 0, s, ws, (uint32_t)shift);
    }
    hipLaunchKernelGGL(k_topk_collect, dim3(blocks), dim3(256), 0, s, d_counts, (uint32_t)n, ws, k);
    hipLaunchKernelGGL(k_topk_sort, dim3(1), dim3(1024), 0, s, ws, k, d_ids, d_vals);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return pfail(TRW_E_DEVICE, std::string("top-k launch: ") + hipGetErrorString(e));
    return TRW_OK;
}

}  // extern "C"
