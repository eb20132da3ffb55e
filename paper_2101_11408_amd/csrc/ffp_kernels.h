// Host-side launchers of the HIP kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "ffp_internal.h"

namespace ffp {

// Bytes per parse tile for tile multiplier k (1, 2 or 4).
int parse_tile_bytes(int k);
hipError_t parse_occupancy(int k, int* blocks_per_cu);

hipError_t launch_init(uint64_t* tile_state, uint64_t ntiles, DeviceState* st,
                       uint64_t* count_out, hipStream_t s);
hipError_t launch_parse(int k, const ParseParams& P, int grid, hipStream_t s);
hipError_t launch_fallback(const FallbackParams& P, int grid, hipStream_t s);

}  // namespace ffp
