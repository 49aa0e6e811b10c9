// Device-side structures of the serving path (shared by the tick kernel and
// the host scheduler).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "trw_internal.hpp"

namespace trw {

constexpr uint32_t kServeBlock = 256;
constexpr uint32_t kChunkQueries = 64;   // queries per ring chunk: one per lane of a wave

// One admitted request, as the tick kernel reads it.
struct ReqDesc {
    uint32_t algo, sampler, max_len, stop_q32;
    uint32_t thr[3];
    uint32_t cancelled;
    uint64_t seed;
    uint64_t qid_base;
    const int32_t *sources;   // arena copy of the request's sources
    int32_t *paths;           // arena: nq rows of `stride` entries
    uint32_t *lengths;        // arena
    uint8_t *status;          // arena
    uint64_t stride;
    uint32_t nq;
    uint32_t pad;
};

// Up to kChunkQueries consecutive queries [begin, end) of request slot `req`.
struct Chunk {
    uint32_t req;
    uint32_t begin;
    uint32_t end;
    uint32_t pad;
};

// A walker slot between ticks.
struct SlotState {
    uint32_t req;     // request slot, or 0xFFFFFFFF when free
    uint32_t qi;
    int32_t cur;
    int32_t prev;
    uint32_t k;
    int32_t off;      // row of cur
    int32_t deg;
    int32_t poff;     // row of prev
    int32_t pdeg;
    int32_t pad[3];
};

// A wave's position in the chunk ring between ticks: the chunk it is
// starting queries from and the one after it, already taken from the ring
// (their sources and row ranges are loaded ahead of need, one query per lane).
struct WaveState {
    unsigned long long claim;   // ring index claimed and not yet read (when has_claim)
    uint32_t req, begin, next, end;         // current chunk: queries [next, end) not yet started
    uint32_t n_req, n_begin, n_end;         // following chunk (n_end == n_begin: none)
    uint32_t has_claim;
    uint32_t pad[2];
};

struct ServeDev {
    ReqDesc *reqs;
    const Chunk *ring;
    uint32_t ring_size;
    unsigned long long *head;          // ring entries claimed (device atomic)
    const unsigned long long *tail;    // ring entries published (written by the host between ticks)
    uint32_t *done;                    // per request slot: queries finished
    unsigned long long *moves;         // moves made, all requests
    SlotState *slots;
    WaveState *waves;
};

hipError_t launch_serve_tick(const GraphDev &g, const TableDev &t, const ServeDev &s, uint32_t steps,
                             uint32_t blocks, hipStream_t stream);

}  // namespace trw
