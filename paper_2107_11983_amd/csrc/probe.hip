// Random-gather probe: the memory system's ceiling for the kind of access a
// walk step makes (a random read whose address depends on the previous read),
// measured on the device itself.  Used as the denominator "achievable random-
// gather bandwidth" next to the HBM peak.
//
// Each lane follows `chains` independent chains for `steps` hops.  A hop reads
// one element of `elem_bytes` (4, 8 or 16) at a pseudo-random index; in the
// dependent form the next index is a hash of the value just read (so the reads
// of one chain serialise, as in a walk), in the independent form it is a hash
// of (lane, hop) only (the throughput ceiling with unlimited parallelism).
//
// Random-scatter probe: the same for writes, the other half of a walk's
// traffic (every query writes its own path row).  Each lane writes `steps`
// elements of `elem_bytes` (16, 64 or 128: one store, a 64-byte block or a
// whole 128-byte cache line, in 16-byte stores) at hashed, element-aligned
// positions.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/trw_probe.h"

namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16; x *= 0x7FEB352Du;
    x ^= x >> 15; x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

__global__ void k_fill(uint32_t *buf, uint64_t n_words, uint32_t seed) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += stride)
        buf[i] = mix32((uint32_t)i ^ seed) ^ (uint32_t)(i >> 32);
}

template <int EB, int CH, bool DEP>
__global__ void __launch_bounds__(256) k_gather(const uint32_t *__restrict__ buf, uint64_t n_elems,
                                                uint32_t steps, uint32_t *__restrict__ sink) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t h[CH];
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) h[c] = mix32(gid * CH + c + 0x9E3779B9u);
    for (uint32_t s = 0; s < steps; ++s) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const uint64_t idx = ((uint64_t)h[c] * n_elems) >> 32;
            uint32_t v;
            if (EB == 16) {
                const uint4 e = reinterpret_cast<const uint4 *>(buf)[idx];
                v = e.x ^ e.y ^ e.z ^ e.w;
            } else if (EB == 8) {
                const uint2 e = reinterpret_cast<const uint2 *>(buf)[idx];
                v = e.x ^ e.y;
            } else {
                v = buf[idx];
            }
            acc += v;
            h[c] = DEP ? mix32(v ^ h[c]) : mix32(h[c] + s + 1);
        }
    }
    if (acc == 0x12345678u) sink[gid & 1023] = acc;   // keeps the loads live
}

template <int EB, int CH>
hipError_t launch_gather(const uint32_t *buf, uint64_t n_elems, uint32_t steps, int dep, uint32_t grid,
                         uint32_t block, uint32_t *sink, hipStream_t s) {
    if (dep)
        hipLaunchKernelGGL((k_gather<EB, CH, true>), dim3(grid), dim3(block), 0, s, buf, n_elems, steps, sink);
    else
        hipLaunchKernelGGL((k_gather<EB, CH, false>), dim3(grid), dim3(block), 0, s, buf, n_elems, steps, sink);
    return hipGetLastError();
}

template <int EB>
hipError_t pick_chains(const uint32_t *buf, uint64_t n_elems, uint32_t steps, uint32_t chains, int dep,
                       uint32_t grid, uint32_t block, uint32_t *sink, hipStream_t s) {
    switch (chains) {
        case 2: return launch_gather<EB, 2>(buf, n_elems, steps, dep, grid, block, sink, s);
        case 4: return launch_gather<EB, 4>(buf, n_elems, steps, dep, grid, block, sink, s);
        default: return launch_gather<EB, 1>(buf, n_elems, steps, dep, grid, block, sink, s);
    }
}

template <int EB>
__global__ void __launch_bounds__(256) k_scatter(uint4 *__restrict__ buf, uint64_t n_elems, uint32_t steps) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t h = mix32(gid + 0x51ED270Bu);
    for (uint32_t s = 0; s < steps; ++s) {
        const uint64_t idx = ((uint64_t)h * n_elems) >> 32;
        uint4 *p = buf + idx * (EB / 16);
#pragma unroll
        for (int j = 0; j < EB / 16; ++j) p[j] = make_uint4(gid, s, (uint32_t)j, h);
        h = mix32(h + s + 1);
    }
}

}  // namespace

extern "C" {

int trw_probe_fill(void *d_buf, uint64_t bytes, uint32_t seed, void *stream) {
    if (!d_buf || bytes < 64 || (reinterpret_cast<uintptr_t>(d_buf) & 15)) return 1;
    hipLaunchKernelGGL(k_fill, dim3(4096), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<uint32_t *>(d_buf), bytes / 4, seed);
    return hipGetLastError() == hipSuccess ? 0 : 3;
}

int trw_probe_gather(const void *d_buf, uint64_t bytes, uint32_t elem_bytes, uint32_t chains, uint32_t steps,
                     int dependent, uint32_t grid, uint32_t block, void *d_sink, void *stream) {
    if (!d_buf || !d_sink || bytes < 64 || (reinterpret_cast<uintptr_t>(d_buf) & 15)) return 1;
    if (!(elem_bytes == 4 || elem_bytes == 8 || elem_bytes == 16)) return 1;
    if (!(chains == 1 || chains == 2 || chains == 4)) return 1;
    if (block == 0 || block > 256 || block % 64 || grid == 0) return 1;
    const uint64_t n_elems = bytes / elem_bytes;
    if (n_elems >= (uint64_t(1) << 32)) return 1;
    auto *buf = static_cast<const uint32_t *>(d_buf);
    auto *sink = static_cast<uint32_t *>(d_sink);
    auto s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (elem_bytes == 16) e = pick_chains<16>(buf, n_elems, steps, chains, dependent, grid, block, sink, s);
    else if (elem_bytes == 8) e = pick_chains<8>(buf, n_elems, steps, chains, dependent, grid, block, sink, s);
    else e = pick_chains<4>(buf, n_elems, steps, chains, dependent, grid, block, sink, s);
    return e == hipSuccess ? 0 : 3;
}

int trw_probe_scatter(void *d_buf, uint64_t bytes, uint32_t elem_bytes, uint32_t steps, uint32_t grid,
                      uint32_t block, void *stream) {
    if (!d_buf || bytes < 128 || (reinterpret_cast<uintptr_t>(d_buf) & 127)) return 1;
    if (!(elem_bytes == 16 || elem_bytes == 64 || elem_bytes == 128)) return 1;
    if (block == 0 || block > 256 || block % 64 || grid == 0) return 1;
    const uint64_t n_elems = bytes / elem_bytes;
    if (n_elems >= (uint64_t(1) << 32)) return 1;
    auto *buf = static_cast<uint4 *>(d_buf);
    auto s = static_cast<hipStream_t>(stream);
    if (elem_bytes == 16) hipLaunchKernelGGL(k_scatter<16>, dim3(grid), dim3(block), 0, s, buf, n_elems, steps);
    else if (elem_bytes == 64) hipLaunchKernelGGL(k_scatter<64>, dim3(grid), dim3(block), 0, s, buf, n_elems, steps);
    else hipLaunchKernelGGL(k_scatter<128>, dim3(grid), dim3(block), 0, s, buf, n_elems, steps);
    return hipGetLastError() == hipSuccess ? 0 : 3;
}

}  // extern "C"
