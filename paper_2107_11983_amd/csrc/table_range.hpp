// Table builds over a vertex range [lo, hi) of a graph view.  Rows of
// vertices outside the range are not built, and the per-vertex outputs (the
// ITS row totals, the REJ bounds p*) are written for the range only; the
// records that carry a destination's row, total or bound read whatever the
// view holds for a destination outside it.  The whole range [0, n) is the
// ordinary build (launch_alias_build and the others).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "trw_internal.hpp"

namespace trw {

struct VRange {
    int64_t lo, hi;
};

hipError_t launch_alias_build_range(const GraphDev &g, int64_t lo, int64_t hi, uint4 *out, hipStream_t s);
hipError_t launch_its_build_range(const GraphDev &g, int64_t lo, int64_t hi, uint64_t *prefix, uint4 *next,
                                  uint64_t *vw, hipStream_t s);
hipError_t launch_rej_build_range(const GraphDev &g, int64_t lo, int64_t hi, uint4 *records, uint32_t *pmax,
                                  hipStream_t s);

}  // namespace trw
