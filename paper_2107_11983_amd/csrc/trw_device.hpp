// Device-side building blocks of the walk engine: the counter-based random
// number generator, integer sampling maps and wavefront helpers.  CDNA4
// (gfx950), wave64.
#pragma once

#if !defined(__HIPCC_RTC__)
#include <hip/hip_runtime.h>
#include <stdint.h>
#else   // runtime compilation (walk programs): the runtime is built in, the integer types namespaced
using __hip_internal::int8_t;
using __hip_internal::int16_t;
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint8_t;
using __hip_internal::uint16_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
typedef unsigned long uintptr_t;
#endif

namespace trw {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two
// 32x32->64 multiplies mixed with the key, the key advancing by the golden-
// ratio Weyl increments between rounds.  Counter = (k, t, qid_lo, qid_hi),
// key = seed, so every query owns a private stream indexed by move and dart.
struct Rand4 {
    uint32_t r0, r1, r2, r3;
};

__device__ __forceinline__ Rand4 philox(uint32_t k, uint32_t t, uint64_t qid, uint64_t seed) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
    uint32_t x0 = k, x1 = t, x2 = (uint32_t)qid, x3 = (uint32_t)(qid >> 32);
    uint32_t ka = (uint32_t)seed, kb = (uint32_t)(seed >> 32);
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        // Each 32x32 -> 64 product as one 64-bit multiply: the compiler then
        // emits one v_mad_u64_u32 for both halves instead of a separate
        // high and low multiply (all quarter-rate).
        const uint64_t pA = (uint64_t)kMulA * x0, pB = (uint64_t)kMulB * x2;
        const uint32_t hiA = (uint32_t)(pA >> 32), loA = (uint32_t)pA;
        const uint32_t hiB = (uint32_t)(pB >> 32), loB = (uint32_t)pB;
        const uint32_t y0 = hiB ^ x1 ^ ka;
        const uint32_t y2 = hiA ^ x3 ^ kb;
        x0 = y0; x1 = loB; x2 = y2; x3 = loA;
        ka += kWeylA; kb += kWeylB;
    }
    return Rand4{x0, x1, x2, x3};
}

// Uniform index in [0, d) from a 32-bit word: the high half of r * d.
__device__ __forceinline__ uint32_t scale32(uint32_t r, uint32_t d) { return __umulhi(r, d); }

// Uniform value in [0, W) from the 64-bit word (r1:r0): the high half of r * W.
__device__ __forceinline__ uint64_t scale64(uint32_t lo, uint32_t hi, uint64_t W) {
    const uint64_t r = ((uint64_t)hi << 32) | lo;
    return __umul64hi(r, W);
}

// ---------------------------------------------------------------------------
// ITS search: the smallest i in [0, d) with x < p[i], where p is a row's
// non-decreasing inclusive prefix (p[d-1] = W > x) and x = high half of
// r64 * W.  The same random fraction scaled to d, g = high half of r64 * d,
// is where a row whose prefix grows evenly has its answer, so the search
// probes g first, gallops outwards (1, 2, 4, ... slots) until the answer is
// bracketed, and finishes by bisection.  With near-uniform weights the
// answer is a few slots from g and the probes share one or two cache lines;
// with skewed weights the gallop costs at most about twice a plain binary
// search.  Any correct search returns the same slot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t its_search(const uint64_t *__restrict__ p, uint32_t d, uint64_t x,
                                               uint64_t r64) {
    const uint32_t g = (uint32_t)__umul64hi(r64, (uint64_t)d);   // < d
    uint32_t lo, hi;                                              // the answer lies in [lo, hi]
    if (x < p[g]) {
        hi = g;
        lo = 0;
        for (uint32_t step = 1; step <= hi; step <<= 1) {
            const uint32_t j = hi - step;
            if (x < p[j]) {
                hi = j;
            } else {
                lo = j + 1;
                break;
            }
        }
    } else {
        lo = g + 1;
        hi = d - 1;
        for (uint32_t step = 1;; step <<= 1) {
            const uint32_t j = lo + step - 1;
            if (j >= d - 1) break;
            if (x < p[j]) {
                hi = j;
                break;
            }
            lo = j + 1;
        }
    }
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (x < p[mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// ITS search by plain bisection over the whole row, with no guess: the
// smallest i in [0, d) with x < p[i] (x < p[d-1] = W).  Same slot as the two
// searches around it; the walks use it for rows below a tuned degree.
__device__ __forceinline__ uint32_t its_bisect(const uint64_t *__restrict__ p, uint32_t d, uint64_t x) {
    uint32_t lo = 0, hi = d - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (x < p[mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// ITS search that starts from the whole 64-byte block around the guess: the
// block's eight prefixes arrive with one round trip and usually bracket the
// answer; otherwise the search gallops outwards from the block's edge and
// ends by bisection.  Same slot as any correct search.  Slots of the block
// outside [0, d) belong to other rows (or to the padding of the prefix
// region, which is rounded up to 256 bytes) and are ignored.
__device__ __forceinline__ uint32_t its_search_block(const uint64_t *__restrict__ p, uint32_t d, uint64_t x,
                                                     uint64_t r64) {
    const uint32_t g = (uint32_t)__umul64hi(r64, (uint64_t)d);   // < d
    const uintptr_t ga = reinterpret_cast<uintptr_t>(p + g);
    const uint4 *blk = reinterpret_cast<const uint4 *>(ga & ~(uintptr_t)63);
    const int32_t b0 = (int32_t)g - (int32_t)((ga & 63) >> 3);    // slot of the block's first prefix
    const uint4 q0 = blk[0], q1 = blk[1], q2 = blk[2], q3 = blk[3];
    const uint64_t v[8] = {(uint64_t)q0.x | ((uint64_t)q0.y << 32), (uint64_t)q0.z | ((uint64_t)q0.w << 32),
                           (uint64_t)q1.x | ((uint64_t)q1.y << 32), (uint64_t)q1.z | ((uint64_t)q1.w << 32),
                           (uint64_t)q2.x | ((uint64_t)q2.y << 32), (uint64_t)q2.z | ((uint64_t)q2.w << 32),
                           (uint64_t)q3.x | ((uint64_t)q3.y << 32), (uint64_t)q3.z | ((uint64_t)q3.w << 32)};
    int32_t lo = -1, hi = (int32_t)d;       // p[lo] <= x (or lo = -1), x < p[hi] (or hi = d)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int32_t i = b0 + j;
        if (i >= 0 && i < (int32_t)d) {
            if (x < v[j]) hi = min(hi, i);
            else lo = max(lo, i);
        }
    }
    if (hi == lo + 1) return (uint32_t)hi;
    if (hi == (int32_t)d) {                  // above the block: gallop up from its last slot
        hi = (int32_t)d - 1;                 // x < p[d - 1] = W
        for (int32_t step = 1;; step <<= 1) {
            const int32_t j = lo + step;
            if (j >= hi) break;
            if (x < p[j]) { hi = j; break; }
            lo = j;
        }
    } else {                                 // below the block: gallop down from its first slot
        for (int32_t step = 1;; step <<= 1) {
            const int32_t j = hi - step;
            if (j <= lo) break;
            if (x < p[j]) hi = j;
            else { lo = j; break; }
        }
    }
    while (hi - lo > 1) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (x < p[mid]) hi = mid; else lo = mid;
    }
    return (uint32_t)hi;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t first_lane_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Wave-aggregated append: lanes with `want` get consecutive slots from *counter.
// Returns this lane's slot (undefined when !want).  One atomic per wave.
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool want) {
    const uint64_t mask = __ballot(want);
    if (mask == 0) return 0;
    const uint32_t total = (uint32_t)__popcll(mask);
    const uint32_t leader = (uint32_t)__builtin_ctzll(mask);
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, total);
    base = __shfl(base, (int)leader);
    return base + rank_below(mask);
}


// Edge hash set of the edge index: open addressing with linear probing from
// SplitMix64's finalizer (Steele, Lea, Flood 2014) of the key u << 32 | v;
// empty slots hold kEsetEmpty (no key has its top bit set: ids are < 2^31).
constexpr unsigned long long kEsetEmpty = ~0ull;

__host__ __device__ inline unsigned long long eset_hash(unsigned long long k) {
    k ^= k >> 30; k *= 0xBF58476D1CE4E5B9ull;
    k ^= k >> 27; k *= 0x94D049BB133111EBull;
    return k ^ (k >> 31);
}

// Is (u, v) in the set?  The set is at most half full, so a probe sequence
// ends at an empty slot.
__device__ __forceinline__ bool eset_has(const unsigned long long *__restrict__ keys, unsigned long long mask,
                                         int32_t u, int32_t v) {
    const unsigned long long key = ((unsigned long long)(uint32_t)u << 32) | (uint32_t)v;
    for (unsigned long long h = eset_hash(key) & mask;; h = (h + 1) & mask) {
        const unsigned long long k = keys[h];
        if (k == key) return true;
        if (k == kEsetEmpty) return false;
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

// The same address as a pointer into global memory.  A pointer read from
// memory (a request's output row, say) is generic, and generic (flat)
// accesses count in both wait counters: a later wait for an LDS exchange or a
// scalar load would then also wait for those stores to reach memory.  Global
// accesses count in the vector-memory counter only.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *global_ptr(T *p) {
    return (__attribute__((address_space(1))) T *)p;
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

    // Last flush of a walk.  The entries after a path's end are unspecified,
    // so the rest of the 64-byte block that holds the last entry is filled
    // (with -1) as far as the row reaches: the block then goes to memory as
    // one whole write rather than a partial one, which HBM has to merge
    // with the old contents.  row_end: one past the row's last entry.  Rows
    // that do not start on 16 bytes (any stride is allowed) get plain writes.
    __device__ __forceinline__ void finish(const int32_t *row_end) {
        if ((reinterpret_cast<uintptr_t>(p) & 15u) != 0 || p + 4 > row_end) {
            flush();
            return;
        }
        if (n > 0) {
            *reinterpret_cast<int4 *>(p) = make_int4(b0, n > 1 ? b1 : -1, n > 2 ? b2 : -1, -1);
            p += 4;
            n = 0;
        }
        while ((reinterpret_cast<uintptr_t>(p) & 63u) != 0 && p + 4 <= row_end) {
            *reinterpret_cast<int4 *>(p) = make_int4(-1, -1, -1, -1);
            p += 4;
        }
    }

    __device__ __forceinline__ void push(int32_t v) {
        if (n == 0) b0 = v; else if (n == 1) b1 = v; else if (n == 2) b2 = v; else b3 = v;
        ++n;
        if (((reinterpret_cast<uintptr_t>(p + n)) & 15u) == 0) flush();
    }
};

}  // namespace trw
