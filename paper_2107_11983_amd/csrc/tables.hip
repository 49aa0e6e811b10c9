// Per-vertex sampling tables (the preprocessing of static walks: the paper
// builds each vertex's table once, before any query runs).
//
// ALIAS: Walker's alias method with Vose's worklist construction in exact
// integers.  The construction pops "small" columns (scaled mass below the row
// total W) and pairs each with the "large" column on top of the large stack,
// both stacks last-in first-out and filled in index order.  Two facts make a
// stack-free, single-pass form possible on the GPU:
//   * a small column is popped exactly once, and the only column whose mass
//     changes is the large column on top; when it falls below W it is pushed
//     on the small stack and therefore popped immediately after;
//   * so the small stack is "the original small columns from the highest
//     index down, with at most one demoted large column in front", and the
//     large stack is "the original large columns from the highest index
//     down".
// Each thread therefore walks its row with two cursors moving downwards and
// keeps one demoted column in registers: O(d) time, O(1) state, no scratch.
//
// ITS: inclusive running sum of the weights per row in uint64.
#include "trw_device.hpp"
#include "trw_internal.hpp"

namespace trw {
namespace {

// floor(s * 2^32 / W) for s < W < 2^63, by restoring shift-subtract division.
__device__ __forceinline__ uint32_t frac32(uint64_t s, uint64_t W) {
    uint64_t rem = s;
    uint32_t q = 0;
#pragma unroll 4
    for (int i = 0; i < 32; ++i) {
        rem <<= 1;
        q <<= 1;
        if (rem >= W) { rem -= W; q |= 1u; }
    }
    return q;
}

// Next index below `from` whose scaled mass w*d is below (want_small) or at least W.
__device__ __forceinline__ int64_t next_below(const uint32_t *__restrict__ w, int64_t from, uint64_t d,
                                              uint64_t W, bool want_small) {
    for (int64_t i = from - 1; i >= 0; --i) {
        const bool small = (uint64_t)w[i] * d < W;
        if (small == want_small) return i;
    }
    return -1;
}

// Row range {row_off, degree} of vertex v.
__device__ __forceinline__ uint2 row_of(const GraphDev &g, int32_t v) {
    const int32_t lo = g.row_ptr[v];
    return make_uint2((uint32_t)lo, (uint32_t)(g.row_ptr[v + 1] - lo));
}

__device__ __forceinline__ void put_entry(uint4 *__restrict__ row, int64_t j, const GraphDev &g, uint32_t thr,
                                          int32_t first, int32_t second) {
    const uint2 a = row_of(g, first), b = row_of(g, second);
    row[2 * j] = make_uint4(thr, (uint32_t)first, (uint32_t)second, 0u);
    row[2 * j + 1] = make_uint4(a.x, a.y, b.x, b.y);
}

__global__ void k_alias_build(GraphDev g, uint4 *__restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    const int64_t off = g.row_ptr[v];
    const int64_t d = (int64_t)g.row_ptr[v + 1] - off;
    if (d <= 0) return;
    const uint32_t *__restrict__ w = g.weight + off;
    const int32_t *__restrict__ col = g.col + off;
    uint4 *__restrict__ row = out + 2 * off;

    uint64_t W = 0;
    for (int64_t i = 0; i < d; ++i) W += w[i];
    if (W == 0) {
        for (int64_t i = 0; i < d; ++i) {
            row[2 * i] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u);
            row[2 * i + 1] = make_uint4(0u, 0u, 0u, 0u);
        }
        return;
    }
    const uint64_t ud = (uint64_t)d;
    int64_t small_next = next_below(w, d, ud, W, true);   // top of the original small stack
    int64_t g_top = next_below(w, d, ud, W, false);       // top of the large stack
    uint64_t g_mass = g_top >= 0 ? (uint64_t)w[g_top] * ud : 0;
    int64_t demoted = -1;                                  // a large column pushed on "small"
    uint64_t demoted_mass = 0;

    while ((demoted >= 0 || small_next >= 0) && g_top >= 0) {
        int64_t l;
        uint64_t l_mass;
        if (demoted >= 0) {
            l = demoted; l_mass = demoted_mass; demoted = -1;
        } else {
            l = small_next; l_mass = (uint64_t)w[l] * ud;
            small_next = next_below(w, l, ud, W, true);
        }
        put_entry(row, l, g, frac32(l_mass, W), col[l], col[g_top]);
        g_mass -= W - l_mass;
        if (g_mass < W) {
            demoted = g_top; demoted_mass = g_mass;
            g_top = next_below(w, g_top, ud, W, false);
            g_mass = g_top >= 0 ? (uint64_t)w[g_top] * ud : 0;
        }
    }
    // Columns left on the large stack are full buckets.
    while (g_top >= 0) {
        put_entry(row, g_top, g, 0xFFFFFFFFu, col[g_top], col[g_top]);
        g_top = next_below(w, g_top, ud, W, false);
    }
}

__global__ void k_its_build(GraphDev g, uint64_t *__restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    const int64_t lo = g.row_ptr[v], hi = g.row_ptr[v + 1];
    uint64_t acc = 0;
    for (int64_t e = lo; e < hi; ++e) {
        acc += g.weight[e];
        out[e] = acc;
    }
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0; }

__global__ void k_validate(GraphDev g, unsigned long long *__restrict__ bad) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > g.n) return;
    unsigned long long nbad = 0;
    if (v == 0 && g.row_ptr[0] != 0) nbad++;
    if (v == g.n) {
        if (g.row_ptr[g.n] != g.m) nbad++;
    } else {
        const int64_t lo = g.row_ptr[v], hi = g.row_ptr[v + 1];
        if (hi < lo || lo < 0 || hi > g.m) {
            nbad++;
        } else {
            int64_t last = -1;
            for (int64_t e = lo; e < hi; ++e) {
                const int64_t c = g.col[e];
                if (c < 0 || c >= g.n || c <= last) nbad++;
                last = c;
            }
        }
    }
    if (nbad) atomicAdd(bad, nbad);
}

// MetaPath label index: stable counting sort of each row by label, one pass
// per label value (O(L * d) per row, L <= kMaxIndexLabels).
__global__ void k_label_index_build(GraphDev g, uint32_t nlab, int32_t *__restrict__ loff,
                                    int32_t *__restrict__ lcol) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    const int64_t off = g.row_ptr[v], end = g.row_ptr[v + 1];
    int32_t *__restrict__ rec = loff + v * (int64_t)(nlab + 1);
    int64_t pos = off;
    for (uint32_t x = 0; x < nlab; ++x) {
        rec[x] = (int32_t)pos;
        for (int64_t e = off; e < end; ++e)
            if (g.label[e] == x) lcol[pos++] = g.col[e];
    }
    rec[nlab] = (int32_t)pos;
    for (; pos < end; ++pos) lcol[pos] = -1;      // edges whose label is >= L
}

// Row-annotated adjacency: every edge slot carries its destination's row
// range, so a walk that picks the slot knows the next row without a lookup.
__global__ void k_adjacency_build(GraphDev g, uint4 *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    const int32_t v = g.col[e];
    const uint2 r = row_of(g, v);
    out[e] = make_uint4((uint32_t)v, r.x, r.y, 0u);
}

// Edges (u, v) whose reverse (v, u) is missing; rows must be sorted.
__global__ void k_symmetry_check(GraphDev g, unsigned long long *__restrict__ bad) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= g.n) return;
    unsigned long long nbad = 0;
    for (int64_t e = g.row_ptr[u]; e < g.row_ptr[u + 1]; ++e) {
        const int32_t v = g.col[e];
        int64_t lo = g.row_ptr[v], hi = g.row_ptr[v + 1];
        bool found = false;
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            const int32_t c = g.col[mid];
            if (c == (int32_t)u) { found = true; break; }
            if (c < (int32_t)u) lo = mid + 1; else hi = mid;
        }
        nbad += !found;
    }
    if (nbad) atomicAdd(bad, nbad);
}

constexpr int kBuildThreads = 256;

}  // namespace

hipError_t launch_alias_build(const GraphDev &g, uint4 *out, hipStream_t s) {
    const int blocks = (g.n + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(k_alias_build, dim3(blocks), dim3(kBuildThreads), 0, s, g, out);
    return hipGetLastError();
}

hipError_t launch_its_build(const GraphDev &g, uint64_t *out, hipStream_t s) {
    const int blocks = (g.n + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(k_its_build, dim3(blocks), dim3(kBuildThreads), 0, s, g, out);
    return hipGetLastError();
}

hipError_t launch_label_index_build(const GraphDev &g, uint32_t nlab, int32_t *loff, int32_t *lcol, hipStream_t s) {
    const int blocks = (g.n + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(k_label_index_build, dim3(blocks), dim3(kBuildThreads), 0, s, g, nlab, loff, lcol);
    return hipGetLastError();
}

hipError_t launch_adjacency_build(const GraphDev &g, uint4 *out, hipStream_t s) {
    const int64_t blocks = ((int64_t)g.m + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(k_adjacency_build, dim3((uint32_t)blocks), dim3(kBuildThreads), 0, s, g, out);
    return hipGetLastError();
}

hipError_t launch_symmetry_check(const GraphDev &g, unsigned long long *d_bad, hipStream_t s) {
    const int blocks = (g.n + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(k_symmetry_check, dim3(blocks), dim3(kBuildThreads), 0, s, g, d_bad);
    return hipGetLastError();
}

hipError_t launch_validate(const GraphDev &g, unsigned long long *d_bad, hipStream_t s) {
    const int blocks = (g.n + 1 + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, d_bad);
    hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(kBuildThreads), 0, s, g, d_bad);
    return hipGetLastError();
}

}  // namespace trw
