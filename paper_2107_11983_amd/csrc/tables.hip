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
// Rows above kBigRow slots get a workgroup each instead (same results): see
// k_alias_build_big.
//
// ITS: inclusive running sum of the weights per row in uint64, then each
// vertex's total and per edge slot a record with the destination's row and
// total (k_its_next).
//
// REJ: the largest weight per row, and per edge slot a record with the
// destination's row and bound (k_rej_records).
#include <algorithm>

#include "table_range.hpp"
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

// Sequential construction of one row by one thread.
__device__ void alias_row_sequential(const GraphDev &g, int64_t off, int64_t d, uint4 *__restrict__ out) {
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

// Rows up to this many slots are built by one thread; longer ones (power-law
// hubs, which would serialise a whole wave or launch) by one workgroup.  On
// R-MAT graphs of average degree 32 the rows above 128 slots are about 3% of
// the rows and hold about 70% of the edges.
constexpr int64_t kBigRow = 128;
constexpr int kBuildBlock = 256;
// Rows above kHugeRow slots (R-MAT's largest hubs, whose one workgroup sets a
// build's time) are built by workgroups of kHugeBlock threads: half the
// block-wide steps, and still no register spills (1024 threads would spill
// the ALIAS build); the tables are the same.
constexpr int64_t kHugeRow = 16384;
constexpr uint32_t kHugeBlock = 512;

__global__ void k_alias_build(GraphDev g, VRange r, uint4 *__restrict__ out) {
    const int64_t v = r.lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= r.hi) return;
    const int64_t off = g.row_ptr[v];
    const int64_t d = (int64_t)g.row_ptr[v + 1] - off;
    if (d <= 0 || d > kBigRow) return;
    alias_row_sequential(g, off, d, out);
}

// Inclusive scan over the NT threads of a workgroup; `total` gets the sum
// over the block.  Every thread must call it.
template <typename T, uint32_t NT = kBuildBlock>
__device__ __forceinline__ T block_inclusive_scan(T v, T *sh, T &total) {
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T t = __shfl_up(v, o);
        if (lane >= (uint32_t)o) v += t;
    }
    if (lane == 63) sh[wv] = v;
    __syncthreads();
    T before = 0;
    total = 0;
#pragma unroll
    for (uint32_t k = 0; k < NT / 64; ++k) {
        if (k < wv) before += sh[k];
        total += sh[k];
    }
    __syncthreads();
    return v + before;
}

template <typename T, uint32_t NT = kBuildBlock>
__device__ __forceinline__ T block_sum(T v, T *sh) {
    T total;
    (void)block_inclusive_scan<T, NT>(v, sh, total);
    return total;
}

// Calls body(v, off, d) for every vertex of [r.lo, r.hi) whose row exceeds
// kBigRow slots, workgroup-uniformly.  Vertices are dealt to the workgroups
// in turn (v - r.lo = j * G + b goes to workgroup b of G), so the hubs, which
// R-MAT numbers first, are spread over the grid instead of falling to one
// workgroup.
// With NT threads per workgroup, the rows of (d_lo, d_hi] slots only.
template <uint32_t NT = kBuildBlock, typename Body>
__device__ __forceinline__ void for_each_big_row(const GraphDev &g, VRange r, int64_t d_lo, int64_t d_hi, Body body) {
    __shared__ uint64_t flags[NT / 64];
    const uint32_t tid = threadIdx.x;
    const int64_t G = gridDim.x;
    for (int64_t base = r.lo; base < r.hi; base += G * NT) {
        const int64_t v = base + (int64_t)tid * G + blockIdx.x;
        const int64_t d = v < r.hi ? (int64_t)g.row_ptr[v + 1] - g.row_ptr[v] : 0;
        const bool big = d > d_lo && d <= d_hi;
        const uint64_t m = __ballot(big);
        if ((tid & 63) == 0) flags[tid >> 6] = m;
        __syncthreads();
        for (uint32_t wv = 0; wv < NT / 64; ++wv) {
            uint64_t bits = flags[wv];
            while (bits) {
                const int64_t u = base + (int64_t)(64 * wv + __builtin_ctzll(bits)) * G + blockIdx.x;
                bits &= bits - 1;
                const int64_t off = g.row_ptr[u];
                body(u, off, (int64_t)g.row_ptr[u + 1] - off);
                __syncthreads();
            }
        }
        __syncthreads();
    }
}
template <typename Body>
__device__ __forceinline__ void for_each_big_row(const GraphDev &g, VRange r, Body body) {
    for_each_big_row<kBuildBlock>(g, r, kBigRow, INT64_MAX, body);
}
template <typename Body>
__device__ __forceinline__ void for_each_big_row(const GraphDev &g, Body body) {
    for_each_big_row(g, VRange{0, g.n}, body);
}

// Virtual 32-bit word k of the scratch area kept in the second 16-byte half of
// a row's entries (that half is written last).
__device__ __forceinline__ uint32_t *scratch_word(uint4 *row, uint64_t k) {
    return reinterpret_cast<uint32_t *>(row) + 8 * (k >> 2) + 4 + (k & 3);
}
__device__ __forceinline__ uint64_t *scratch_u64(uint4 *row, uint64_t k) {   // k even
    return reinterpret_cast<uint64_t *>(scratch_word(row, k));
}

// ALIAS for a long row, one workgroup, same result as the worklist procedure.
// Number the original small columns in the order they are popped (descending
// index) l_1, l_2, ..., with deficits W - s and prefix sums D_0 = 0, D_1, ...;
// and the large columns likewise g_1, g_2, ... with surpluses s - W and prefix
// sums S_1, S_2, ... (exact integers: D_total = S_total).  Deficits are charged
// to the large columns in order, a large column being demoted once the charges
// exceed its surplus, and a demoted column passes its excess on to the next.
// Hence:
//   * l_i is paired with the top of the large stack when it is popped,
//     g_J with J = min{j : S_j >= D_(i-1)};
//   * g_j with S_j >= D_total is never demoted (a full bucket);
//   * otherwise g_j is demoted while serving l_i, i = min{i : D_i > S_j}, keeps
//     mass W - (D_i - S_j) and is paired with the next large column g_(j+1).
// Both prefix sums come from block scans; every bucket is then independent.
//
// Scratch words: [0, n_s) small indices in pop order, [n_s, d) large indices
// in pop order, then (at an even word) the u64 array P with P[0] = 0,
// P[1..n_s] = D, P[n_s+1 .. n_s+n_l] = S.  3d + 3 words fit in the 4d words
// of the second halves for d > 3.
template <uint32_t NT>
__global__ void __launch_bounds__(NT) k_alias_build_big(GraphDev g, VRange r, int64_t d_lo, int64_t d_hi,
                                                  uint4 *__restrict__ out) {
    __shared__ uint64_t sh64[NT / 64];
    __shared__ uint32_t sh32[NT / 64];
    const uint32_t tid = threadIdx.x;
    for_each_big_row<NT>(g, r, d_lo, d_hi, [&](int64_t v, int64_t off, int64_t d) {
        const uint32_t *__restrict__ w = g.weight + off;
        const int32_t *__restrict__ col = g.col + off;
        uint4 *__restrict__ row = out + 2 * off;
        const uint64_t ud = (uint64_t)d;
        (void)v;

        uint64_t part = 0;
        for (int64_t i = tid; i < d; i += NT) part += w[i];
        const uint64_t W = block_sum<uint64_t, NT>(part, sh64);
        if (W == 0 || W > ~0ull / ud) {                        // no transition, or d*W would overflow
            if (tid == 0) alias_row_sequential(g, off, d, out);
            return;
        }
        uint32_t cs = 0;
        for (int64_t i = tid; i < d; i += NT) cs += ((uint64_t)w[i] * ud < W);
        const uint64_t n_s = block_sum<uint32_t, NT>(cs, sh32);
        const uint64_t n_l = ud - n_s;
        const uint64_t pbase = ud + (ud & 1);
        if (tid == 0) *scratch_u64(row, pbase) = 0;
        uint64_t carry_s = 0, carry_l = 0, carry_D = 0, carry_S = 0;
        for (int64_t r0 = 0; r0 < d; r0 += NT) {
            const int64_t r = r0 + tid;                        // position in descending index order
            const bool in = r < d;
            const int64_t i = d - 1 - r;
            const uint64_t s_i = in ? (uint64_t)w[i] * ud : 0;
            const bool small = in && s_i < W;
            const bool large = in && !small;
            uint32_t ts, tl;
            uint64_t tD, tS;
            const uint32_t is = block_inclusive_scan<uint32_t, NT>((uint32_t)small, sh32, ts);
            const uint32_t il = block_inclusive_scan<uint32_t, NT>((uint32_t)large, sh32, tl);
            const uint64_t iD = block_inclusive_scan<uint64_t, NT>(small ? W - s_i : 0ull, sh64, tD);
            const uint64_t iS = block_inclusive_scan<uint64_t, NT>(large ? s_i - W : 0ull, sh64, tS);
            if (small) {
                const uint64_t pos = carry_s + is - 1;
                *scratch_word(row, pos) = (uint32_t)i;
                *scratch_u64(row, pbase + 2 * (pos + 1)) = carry_D + iD;
            } else if (large) {
                const uint64_t pos = carry_l + il - 1;
                *scratch_word(row, n_s + pos) = (uint32_t)i;
                *scratch_u64(row, pbase + 2 * (n_s + 1 + pos)) = carry_S + iS;
            }
            carry_s += ts; carry_l += tl; carry_D += tD; carry_S += tS;
        }
        __syncthreads();
        const uint64_t D_total = carry_D;
        for (uint64_t pos = tid; pos < n_s; pos += NT) {       // small columns
            const uint32_t l = *scratch_word(row, pos);
            const uint64_t x = *scratch_u64(row, pbase + 2 * pos);   // D_(i-1)
            uint64_t lo = 0, hi = n_l - 1;
            while (lo < hi) {
                const uint64_t mid = (lo + hi) >> 1;
                if (*scratch_u64(row, pbase + 2 * (n_s + 1 + mid)) >= x) hi = mid; else lo = mid + 1;
            }
            const uint32_t gl = *scratch_word(row, n_s + lo);
            row[2 * l] = make_uint4(frac32((uint64_t)w[l] * ud, W), (uint32_t)col[l], (uint32_t)col[gl], 0u);
        }
        for (uint64_t pos = tid; pos < n_l; pos += NT) {       // large columns
            const uint32_t gl = *scratch_word(row, n_s + pos);
            const uint64_t S = *scratch_u64(row, pbase + 2 * (n_s + 1 + pos));
            if (S >= D_total) {
                row[2 * gl] = make_uint4(0xFFFFFFFFu, (uint32_t)col[gl], (uint32_t)col[gl], 0u);
            } else {
                uint64_t lo = 1, hi = n_s;
                while (lo < hi) {
                    const uint64_t mid = (lo + hi) >> 1;
                    if (*scratch_u64(row, pbase + 2 * mid) > S) hi = mid; else lo = mid + 1;
                }
                const uint64_t Di = *scratch_u64(row, pbase + 2 * lo);
                const uint32_t nx = *scratch_word(row, n_s + pos + 1);
                row[2 * gl] = make_uint4(frac32(W - (Di - S), W), (uint32_t)col[gl], (uint32_t)col[nx], 0u);
            }
        }
        __syncthreads();
        for (int64_t j = tid; j < d; j += NT) {                // second halves, over the scratch
            const uint4 e = row[2 * j];
            const uint2 ra = row_of(g, (int32_t)e.y), rb = row_of(g, (int32_t)e.z);
            row[2 * j + 1] = make_uint4(ra.x, ra.y, rb.x, rb.y);
        }
    });
}

__global__ void k_its_build(GraphDev g, VRange r, uint64_t *__restrict__ out) {
    const int64_t v = r.lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= r.hi) return;
    const int64_t lo = g.row_ptr[v], hi = g.row_ptr[v + 1];
    if (hi - lo > kBigRow) return;
    uint64_t acc = 0;
    for (int64_t e = lo; e < hi; ++e) {
        acc += g.weight[e];
        out[e] = acc;
    }
}

template <uint32_t NT>
__global__ void __launch_bounds__(NT) k_its_build_big(GraphDev g, VRange r, int64_t d_lo, int64_t d_hi,
                                                uint64_t *__restrict__ out) {
    __shared__ uint64_t sh64[NT / 64];
    for_each_big_row<NT>(g, r, d_lo, d_hi, [&](int64_t, int64_t off, int64_t d) {
        uint64_t carry = 0;
        for (int64_t r0 = 0; r0 < d; r0 += NT) {
            const int64_t e = off + r0 + threadIdx.x;
            const bool in = r0 + threadIdx.x < d;
            uint64_t tot;
            const uint64_t inc = block_inclusive_scan<uint64_t, NT>(in ? (uint64_t)g.weight[e] : 0ull, sh64, tot);
            if (in) out[e] = carry + inc;
            carry += tot;
        }
    });
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
        } else if (hi - lo <= kBigRow) {     // longer rows: k_validate_big
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

// The slots of rows above kBigRow (whose row ranges k_validate has checked),
// a workgroup per row: in range and strictly increasing.
__global__ void __launch_bounds__(kBuildBlock) k_validate_big(GraphDev g, unsigned long long *__restrict__ bad) {
    unsigned long long nbad = 0;
    for_each_big_row(g, [&](int64_t, int64_t off, int64_t d) {
        const int64_t hi = off + d;
        if (off < 0 || hi > g.m) return;                       // reported by k_validate
        for (int64_t e = off + threadIdx.x; e < hi; e += kBuildBlock) {
            const int64_t c = g.col[e];
            if (c < 0 || c >= g.n || (e > off && c <= (int64_t)g.col[e - 1])) nbad++;
        }
    });
    if (nbad) atomicAdd(bad, nbad);
}

// MetaPath label index: stable counting sort of each row by label, one pass
// per label value (O(L * d) per row, L <= kMaxIndexLabels); a thread per row
// up to kBigRow slots, a workgroup with block scans above.
__global__ void k_label_index_build(GraphDev g, uint32_t nlab, int32_t *__restrict__ loff,
                                    int32_t *__restrict__ lcol) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    const int64_t off = g.row_ptr[v], end = g.row_ptr[v + 1];
    if (end - off > kBigRow) return;
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

// Fused entries (L <= kMaxFusedLabels): slot e of the label-sorted rows holds
// its destination and that vertex's L + 1 label offsets, so a MetaPath move
// reads one 32-byte entry that also tells the next move where its label's run
// is.  Slots of edges left out of the index (label >= L) hold destination -1.
__global__ void k_label_fused(GraphDev g, uint32_t nlab, const int32_t *__restrict__ loff,
                              const int32_t *__restrict__ lcol, uint4 *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    const int32_t v = lcol[e];
    int32_t o[kMaxFusedLabels + 1] = {0, 0, 0, 0, 0, 0, 0};
    if (v >= 0 && v < g.n) {
        const int32_t *rec = loff + (int64_t)v * (nlab + 1);
#pragma unroll
        for (uint32_t i = 0; i <= kMaxFusedLabels; ++i)
            if (i <= nlab) o[i] = rec[i];
    }
    out[2 * e] = make_uint4((uint32_t)v, (uint32_t)o[0], (uint32_t)o[1], (uint32_t)o[2]);
    out[2 * e + 1] = make_uint4((uint32_t)o[3], (uint32_t)o[4], (uint32_t)o[5], (uint32_t)o[6]);
}

__global__ void __launch_bounds__(kBuildBlock) k_label_index_build_big(GraphDev g, uint32_t nlab,
                                                                       int32_t *__restrict__ loff,
                                                                       int32_t *__restrict__ lcol) {
    __shared__ uint32_t sh32[kBuildBlock / 64];
    for_each_big_row(g, [&](int64_t v, int64_t off, int64_t d) {
        const int64_t end = off + d;
        int32_t *__restrict__ rec = loff + v * (int64_t)(nlab + 1);
        int64_t pos = off;
        for (uint32_t x = 0; x < nlab; ++x) {
            if (threadIdx.x == 0) rec[x] = (int32_t)pos;
            for (int64_t e0 = off; e0 < end; e0 += kBuildBlock) {
                const int64_t e = e0 + threadIdx.x;
                const bool hit = e < end && g.label[e] == x;
                uint32_t tot;
                const uint32_t inc = block_inclusive_scan((uint32_t)hit, sh32, tot);
                if (hit) lcol[pos + inc - 1] = g.col[e];
                pos += tot;
            }
        }
        if (threadIdx.x == 0) rec[nlab] = (int32_t)pos;
        for (int64_t e = pos + threadIdx.x; e < end; e += kBuildBlock) lcol[e] = -1;
    });
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

// ITS next records: per vertex its weight sum W (the last prefix of its row),
// and per edge slot the destination's id, row range and W, so that a move is
// the search over the prefix plus one 32-byte read, with no lookup of the
// chosen slot's destination, its row or its total:
//   [0] {dst, row_off(dst), deg(dst), 0}   [1] {W(dst) lo, W(dst) hi, 0, 0}
__global__ void k_its_vw(GraphDev g, VRange r, const uint64_t *__restrict__ prefix, uint64_t *__restrict__ vw) {
    const int64_t v = r.lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= r.hi) return;
    const int64_t hi = g.row_ptr[v + 1];
    vw[v] = hi > g.row_ptr[v] ? prefix[hi - 1] : 0ull;
}

__global__ void k_its_next(GraphDev g, const uint64_t *__restrict__ vw, uint4 *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    const int32_t v = g.col[e];
    const uint2 r = row_of(g, v);
    const uint64_t W = vw[v];
    out[2 * e] = make_uint4((uint32_t)v, r.x, r.y, 0u);
    out[2 * e + 1] = make_uint4((uint32_t)W, (uint32_t)(W >> 32), 0u, 0u);
}

// REJ (rejection sampling): the initialization finds p*_v, the largest
// weight of v's row, kept per vertex after the slot records.  Every slot's
// record then carries its weight and the destination's id, row range and
// p*, so a dart is one 32-byte read and a hit needs no further lookup:
//   [0] {w, dst, row_off(dst), deg(dst)}   [1] {p*(dst), 0, 0, 0}
__global__ void k_rej_pmax(GraphDev g, VRange r, uint32_t *__restrict__ pmax) {
    const int64_t v = r.lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= r.hi) return;
    const int64_t lo = g.row_ptr[v], hi = g.row_ptr[v + 1];
    if (hi - lo > kBigRow) return;
    uint32_t mx = 0;
    for (int64_t e = lo; e < hi; ++e) mx = max(mx, g.weight[e]);
    pmax[v] = mx;
}

__global__ void __launch_bounds__(kBuildBlock) k_rej_pmax_big(GraphDev g, VRange r, uint32_t *__restrict__ pmax) {
    __shared__ uint32_t sh[kBuildBlock / 64];
    for_each_big_row(g, r, [&](int64_t v, int64_t off, int64_t d) {
        uint32_t mx = 0;
        for (int64_t e = off + threadIdx.x; e < off + d; e += kBuildBlock) mx = max(mx, g.weight[e]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o));
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t m = 0;
            for (uint32_t i = 0; i < kBuildBlock / 64; ++i) m = max(m, sh[i]);
            pmax[v] = m;
        }
    });
}

__global__ void k_rej_records(GraphDev g, const uint32_t *__restrict__ pmax, uint4 *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    const int32_t v = g.col[e];
    const uint2 r = row_of(g, v);
    out[2 * e] = make_uint4(g.weight[e], (uint32_t)v, r.x, r.y);
    out[2 * e + 1] = make_uint4(pmax[v], 0u, 0u, 0u);
}

// Edge hash set (the edge index's membership test for Node2Vec): every edge
// (u, v) inserted once as u << 32 | v by compare-and-swap with linear
// probing; a thread per row up to kBigRow slots, a workgroup per longer row.
__global__ void k_fill_u64(unsigned long long *p, unsigned long long n, unsigned long long v) {
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__device__ __forceinline__ void eset_insert(unsigned long long *keys, unsigned long long mask, unsigned long long key) {
    for (unsigned long long h = eset_hash(key) & mask;; h = (h + 1) & mask) {
        const unsigned long long old = atomicCAS(&keys[h], kEsetEmpty, key);
        if (old == kEsetEmpty || old == key) return;
    }
}

__global__ void k_edge_set_build(GraphDev g, unsigned long long *keys, unsigned long long mask) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= g.n) return;
    const int64_t lo = g.row_ptr[u], hi = g.row_ptr[u + 1];
    if (hi - lo > kBigRow) return;
    for (int64_t e = lo; e < hi; ++e)
        eset_insert(keys, mask, ((unsigned long long)u << 32) | (uint32_t)g.col[e]);
}

__global__ void __launch_bounds__(kBuildBlock) k_edge_set_build_big(GraphDev g, unsigned long long *keys,
                                                                    unsigned long long mask) {
    for_each_big_row(g, [&](int64_t u, int64_t off, int64_t d) {
        for (int64_t e = off + threadIdx.x; e < off + d; e += kBuildBlock)
            eset_insert(keys, mask, ((unsigned long long)u << 32) | (uint32_t)g.col[e]);
    });
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

// Workgroups for the big-row kernels: one per vertex up to 2048 (each deals
// itself every G-th vertex).
int big_row_blocks(int64_t verts) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(verts, 2048));
}
int big_row_blocks(const GraphDev &g) { return big_row_blocks((int64_t)g.n); }
// Workgroups for the huge-row kernels (few rows, each a long loop).
int huge_row_blocks(int64_t verts) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(verts, 512));
}

// Thread-per-vertex workgroups for [lo, hi) (at least one).
int vertex_blocks(VRange r) {
    return (int)std::max<int64_t>(1, (r.hi - r.lo + kBuildThreads - 1) / kBuildThreads);
}

}  // namespace

hipError_t launch_alias_build_range(const GraphDev &g, int64_t lo, int64_t hi, uint4 *out, hipStream_t s) {
    const VRange r{lo, hi};
    hipLaunchKernelGGL(k_alias_build, dim3(vertex_blocks(r)), dim3(kBuildThreads), 0, s, g, r, out);
    hipLaunchKernelGGL(k_alias_build_big<kBuildBlock>, dim3(big_row_blocks(hi - lo)), dim3(kBuildBlock), 0, s, g, r,
                       kBigRow, kHugeRow, out);
    hipLaunchKernelGGL(k_alias_build_big<kHugeBlock>, dim3(huge_row_blocks(hi - lo)), dim3(kHugeBlock), 0, s, g, r,
                       kHugeRow, INT64_MAX, out);
    return hipGetLastError();
}

hipError_t launch_alias_build(const GraphDev &g, uint4 *out, hipStream_t s) {
    return launch_alias_build_range(g, 0, g.n, out, s);
}

hipError_t launch_its_build_range(const GraphDev &g, int64_t lo, int64_t hi, uint64_t *prefix, uint4 *next,
                                  uint64_t *vw, hipStream_t s) {
    const VRange r{lo, hi};
    if (g.m > 0) {
        hipLaunchKernelGGL(k_its_build, dim3(vertex_blocks(r)), dim3(kBuildThreads), 0, s, g, r, prefix);
        hipLaunchKernelGGL(k_its_build_big<kBuildBlock>, dim3(big_row_blocks(hi - lo)), dim3(kBuildBlock), 0, s, g, r,
                           kBigRow, kHugeRow, prefix);
        hipLaunchKernelGGL(k_its_build_big<kHugeBlock>, dim3(huge_row_blocks(hi - lo)), dim3(kHugeBlock), 0, s, g,
                           r, kHugeRow, INT64_MAX, prefix);
    }
    hipLaunchKernelGGL(k_its_vw, dim3(vertex_blocks(r)), dim3(kBuildThreads), 0, s, g, r, prefix, vw);
    if (g.m > 0) {
        const int64_t eblocks = ((int64_t)g.m + kBuildThreads - 1) / kBuildThreads;
        hipLaunchKernelGGL(k_its_next, dim3((uint32_t)eblocks), dim3(kBuildThreads), 0, s, g, vw, next);
    }
    return hipGetLastError();
}

hipError_t launch_its_build(const GraphDev &g, uint64_t *prefix, uint4 *next, uint64_t *vw, hipStream_t s) {
    return launch_its_build_range(g, 0, g.n, prefix, next, vw, s);
}

hipError_t launch_label_fused_build(const GraphDev &g, uint32_t nlab, const int32_t *loff, const int32_t *lcol,
                                    uint4 *out, hipStream_t s) {
    const int64_t eblocks = ((int64_t)g.m + kBuildThreads - 1) / kBuildThreads;
    if (eblocks > 0)
        hipLaunchKernelGGL(k_label_fused, dim3((uint32_t)eblocks), dim3(kBuildThreads), 0, s, g, nlab, loff, lcol, out);
    return hipGetLastError();
}

hipError_t launch_label_index_build(const GraphDev &g, uint32_t nlab, int32_t *loff, int32_t *lcol, hipStream_t s) {
    const int blocks = (g.n + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(k_label_index_build, dim3(blocks), dim3(kBuildThreads), 0, s, g, nlab, loff, lcol);
    hipLaunchKernelGGL(k_label_index_build_big, dim3(big_row_blocks(g)), dim3(kBuildBlock), 0, s, g, nlab, loff,
                       lcol);
    return hipGetLastError();
}

hipError_t launch_adjacency_build(const GraphDev &g, uint4 *out, hipStream_t s) {
    const int64_t blocks = ((int64_t)g.m + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(k_adjacency_build, dim3((uint32_t)blocks), dim3(kBuildThreads), 0, s, g, out);
    return hipGetLastError();
}

hipError_t launch_rej_build_range(const GraphDev &g, int64_t lo, int64_t hi, uint4 *records, uint32_t *pmax,
                                  hipStream_t s) {
    const VRange r{lo, hi};
    hipLaunchKernelGGL(k_rej_pmax, dim3(vertex_blocks(r)), dim3(kBuildThreads), 0, s, g, r, pmax);
    hipLaunchKernelGGL(k_rej_pmax_big, dim3(big_row_blocks(hi - lo)), dim3(kBuildBlock), 0, s, g, r, pmax);
    if (g.m > 0) {
        const int64_t eblocks = ((int64_t)g.m + kBuildThreads - 1) / kBuildThreads;
        hipLaunchKernelGGL(k_rej_records, dim3((uint32_t)eblocks), dim3(kBuildThreads), 0, s, g, pmax, records);
    }
    return hipGetLastError();
}

hipError_t launch_rej_build(const GraphDev &g, uint4 *records, uint32_t *pmax, hipStream_t s) {
    return launch_rej_build_range(g, 0, g.n, records, pmax, s);
}

hipError_t launch_edge_set_build(const GraphDev &g, unsigned long long *keys, unsigned long long slots, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3(4096), dim3(256), 0, s, keys, slots, kEsetEmpty);
    const int blocks = (g.n + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(k_edge_set_build, dim3(blocks), dim3(kBuildThreads), 0, s, g, keys, slots - 1);
    hipLaunchKernelGGL(k_edge_set_build_big, dim3(big_row_blocks(g)), dim3(kBuildBlock), 0, s, g, keys, slots - 1);
    return hipGetLastError();
}

hipError_t launch_symmetry_check(const GraphDev &g, unsigned long long *d_bad, hipStream_t s) {
    const int blocks = (g.n + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(k_symmetry_check, dim3(blocks), dim3(kBuildThreads), 0, s, g, d_bad);
    return hipGetLastError();
}

// Sources outside [0, n): a grid-stride count, summed per wave, one atomic per
// wave.  At most 4096 x 256 threads, so a wave's sum of its lanes' counts
// (each below 2^32 / 2^20 = 4096) fits 32 bits.
__global__ void __launch_bounds__(256) k_count_bad_sources(const int32_t *__restrict__ src, uint64_t nq, int32_t n,
                                                           unsigned long long *__restrict__ bad) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t nbad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += stride)
        nbad += (uint32_t)src[i] >= (uint32_t)n ? 1u : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nbad += __shfl_xor(nbad, o);
    if ((threadIdx.x & 63) == 0 && nbad) atomicAdd(bad, (unsigned long long)nbad);
}

hipError_t launch_validate_sources(const int32_t *src, uint64_t nq, int32_t n, unsigned long long *d_bad,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, d_bad);
    if (nq > 0) {
        const uint64_t blocks = std::min<uint64_t>((nq + 255) / 256, 4096);
        hipLaunchKernelGGL(k_count_bad_sources, dim3((uint32_t)blocks), dim3(256), 0, s, src, nq, n, d_bad);
    }
    return hipGetLastError();
}

hipError_t launch_validate(const GraphDev &g, unsigned long long *d_bad, hipStream_t s) {
    const int blocks = (g.n + 1 + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, d_bad);
    hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(kBuildThreads), 0, s, g, d_bad);
    hipLaunchKernelGGL(k_validate_big, dim3(big_row_blocks(g)), dim3(kBuildBlock), 0, s, g, d_bad);
    return hipGetLastError();
}

}  // namespace trw
