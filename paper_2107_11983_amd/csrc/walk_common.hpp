// Device pieces shared by the batch walk kernels and the serving tick.
#pragma once

#include "trw_device.hpp"
#include "trw_internal.hpp"

namespace trw {

constexpr uint32_t kIdle = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t wave_total(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---------------------------------------------------------------------------
// Move of a static walk that reads the adjacency array (NAIVE, ITS).  Returns
// the next vertex, or -1 when the row has no transition (weights sum to 0).
// ---------------------------------------------------------------------------
template <uint32_t SMP>
__device__ __forceinline__ int32_t static_next(const GraphDev &g, const TableDev &t, int32_t off, uint32_t d,
                                               const Rand4 &r, uint32_t gallop_min) {
    if (SMP == SMP_NAIVE) return g.col[off + scale32(r.r0, d)];
    // ITS: x uniform in [0, W) from 64 bits, smallest i with x < prefix[i];
    // rows of at least gallop_min slots search from the guess, shorter ones bisect
    const uint64_t *__restrict__ p = t.prefix + off;
    const uint64_t W = p[d - 1];
    if (W == 0) return -1;
    const uint64_t x = scale64(r.r0, r.r1, W);
    const uint32_t i = d >= gallop_min ? its_search(p, d, x, ((uint64_t)r.r1 << 32) | r.r0) : its_bisect(p, d, x);
    return g.col[off + i];
}

// ---------------------------------------------------------------------------
// REJ (Sampling Methods, rejection sampling): a dart (x, y) has x a uniform
// edge slot of cur and y = r1 * p*(cur) / 2^32 uniform in [0, p*); it hits
// iff y < w_x, i.e. r1 * p* < w_x * 2^32 in exact 64-bit integers.  Dart t of
// move k uses Philox block (k, t); the hitting dart's block also gives PPR's
// stop coin.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool rej_hit(uint32_t r1, uint32_t pmax, uint32_t w) {
    return (uint64_t)r1 * pmax < ((uint64_t)w << 32);
}

// Throws darts until one hits (the per-step schedule; the persistent kernel
// throws one dart per iteration instead).  r holds dart 0's block on entry
// and the hitting dart's block on return.  Returns the next vertex and its
// row and p*, or -1 when cur has no transition (p* == 0).
__device__ __forceinline__ int32_t rej_move(const TableDev &t, const WalkDev &a, uint64_t qid, uint32_t k,
                                            int32_t off, uint32_t d, uint32_t pm, Rand4 &r, int32_t &noff,
                                            int32_t &ndeg, uint32_t &npm) {
    if (pm == 0) return -1;
    for (uint32_t dart = 0;; ++dart) {
        if (dart > 0) r = philox(k, dart, qid, a.seed);
        const uint64_t e = (uint64_t)(uint32_t)off + scale32(r.r0, d);
        const uint4 rec = t.rej[2 * e];
        if (rej_hit(r.r1, pm, rec.x) || dart + 1 == kMaxDarts) {
            noff = (int32_t)rec.z;
            ndeg = (int32_t)rec.w;
            npm = t.rej[2 * e + 1].x;
            return (int32_t)rec.y;
        }
    }
}

// ---------------------------------------------------------------------------
// Node2Vec move, O-REJ (Sampling Methods: rejection with a user bound p*):
// throw darts (x, y) with x a uniform edge slot of cur and y = r1 >> 16 until
// y falls under the Q16 threshold of x's class (x == prev, x adjacent to
// prev, otherwise; the Node2Vec transition equation).  The adjacency test is
// a binary search in a sorted row, or a probe of the edge index's hash set,
// made only when the dart's height lies between the two thresholds it would
// choose between.  With the adjacency
// index a dart also learns x's row, so on a symmetric graph the search can run
// in the shorter of the two rows (x in N(prev) iff prev in N(x)), and an
// accepted move needs no row lookup.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool in_row(const int32_t *__restrict__ col, int32_t lo, int32_t hi, int32_t key) {
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        const int32_t c = col[mid];
        if (c == key) return true;
        if (c < key) lo = mid + 1; else hi = mid;
    }
    return false;
}

// FIRST: the caller has already read the first dart's adjacency record
// (slot off + scale32(r.r0, d)) and passes it as `first`.
template <bool ADJ, bool FIRST = false>
__device__ __forceinline__ int32_t n2v_move(const GraphDev &g, const TableDev &t, const WalkDev &a, uint64_t qid,
                                            uint32_t k, int32_t off, uint32_t d, const Rand4 &r, int32_t prev,
                                            int32_t poff, int32_t pd, int32_t &noff, int32_t &ndeg,
                                            const uint4 &first = uint4{}) {
    Rand4 rr = r;
    for (uint32_t dart = 0;; ++dart) {
        if (dart > 0) rr = philox(k, dart, qid, a.seed);
        const uint32_t slot = (uint32_t)off + scale32(rr.r0, d);
        int32_t x, xo = 0, xd = 0;
        if (ADJ) {
            const uint4 e = (FIRST && dart == 0) ? first : t.adj[slot];
            x = (int32_t)e.x; xo = (int32_t)e.y; xd = (int32_t)e.z;
        } else {
            x = g.col[slot];
        }
        bool accept = (k == 0 || dart + 1 == kMaxDarts);
        if (!accept) {
            const uint32_t y = rr.r1 >> 16;
            if (x == prev) {
                accept = y < a.thr[0];
            } else if (y < min(a.thr[1], a.thr[2])) {
                accept = true;          // under both thresholds: the adjacency test cannot change it
            } else if (y >= max(a.thr[1], a.thr[2])) {
                accept = false;         // over both
            } else {
                bool adjacent;
                if (t.eset && (uint32_t)pd > a.n2v_search) {   // edge index: one probe sequence, usually one line
                    adjacent = eset_has(t.eset, t.eset_mask, prev, x);
                } else if (t.eset) {        // a short row of prev: search it (a tuned degree)
                    adjacent = in_row(g.col, poff, poff + pd, x);
                } else {
                    adjacent = (ADJ && g.symmetric && xd < pd) ? in_row(g.col, xo, xo + xd, prev)
                                                               : in_row(g.col, poff, poff + pd, x);
                }
                accept = y < (adjacent ? a.thr[1] : a.thr[2]);
            }
        }
        if (accept) {
            noff = xo; ndeg = xd;
            return x;
        }
    }
}

}  // namespace trw
