// Device-side building blocks of the walk engine: the counter-based random
// number generator, integer sampling maps and wavefront helpers.  CDNA4
// (gfx950), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
        const uint32_t hiA = __umulhi(kMulA, x0), loA = kMulA * x0;
        const uint32_t hiB = __umulhi(kMulB, x2), loB = kMulB * x2;
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

}  // namespace trw
