/*
 * trw_probe.h — measurement probe exported by libtrw.so (not part of the walk
 * path).  It measures the rate at which the GPU serves random reads of the
 * kind a walk step makes, giving the "achievable random-gather bandwidth"
 * that the walk's throughput is compared with beside the HBM peak.  The paper
 * makes the same comparison on its CPU: the memory bandwidth its walks reach
 * against the machine's measured maximum (Motivations, Observations).
 *
 * Return values: 0 ok, 1 invalid argument, 3 HIP launch error.
 * Both calls are asynchronous on `stream` (a hipStream_t).
 */
#ifndef TRW_PROBE_H
#define TRW_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Fill `bytes` of device memory at d_buf (16-byte aligned) with hashed words. */
int trw_probe_fill(void *d_buf, uint64_t bytes, uint32_t seed, void *stream);

/*
 * grid x block lanes each follow `chains` (1, 2 or 4) chains of `steps`
 * random reads of `elem_bytes` (4, 8 or 16) from the `bytes`-long buffer
 * d_buf (bytes / elem_bytes < 2^32).  dependent != 0: each read's index is a
 * hash of the previous value (serial chain); 0: a hash of (lane, step) only.
 * d_sink: device scratch of at least 4096 bytes (written only to keep the
 * loads live).  block: 64..256, a multiple of 64.
 */
int trw_probe_gather(const void *d_buf, uint64_t bytes, uint32_t elem_bytes, uint32_t chains, uint32_t steps,
                     int dependent, uint32_t grid, uint32_t block, void *d_sink, void *stream);

/*
 * grid x block lanes each write `steps` elements of `elem_bytes` (16, 64 or
 * 128, written as 16-byte stores) at hashed, element-aligned positions of the
 * `bytes`-long buffer d_buf (128-byte aligned, bytes / elem_bytes < 2^32).
 * The random-write counterpart of trw_probe_gather: a walk writes one path
 * row per query.  block: 64..256, a multiple of 64.
 */
int trw_probe_scatter(void *d_buf, uint64_t bytes, uint32_t elem_bytes, uint32_t steps, uint32_t grid,
                      uint32_t block, void *stream);

/*
 * Replay a request trace against a server (trw.h): request i (trw_request) is
 * submitted once arrival_ns[i] nanoseconds (non-decreasing) have passed since
 * the call began, and its completion is stored in completions[i]
 * (trw_completion).  Runs in the calling thread until all n complete.
 * Returns 0, 1 (bad argument), 6 (timeout_ms passed), 10 + a trw_status from
 * submit, or 20 + a trw_status from poll.
 */
int trw_probe_serve_replay(void *server, uint32_t n, const void *requests, const uint64_t *arrival_ns,
                           void *completions, uint32_t timeout_ms);

#ifdef __cplusplus
}
#endif

#endif /* TRW_PROBE_H */
