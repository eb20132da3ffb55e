// Host-side launchers of the HIP kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "ffp_internal.h"

namespace ffp {

// Bytes per parse tile for tile multiplier k (1, 2 or 4).
int parse_tile_bytes(int k);
// Resident workgroups per CU of the parse kernel: of the plain instance
// without a reduction, or (wide) of the largest of the other instances.
hipError_t parse_occupancy(int k, bool single_delim, bool wide, int* blocks_per_cu);

// Device address of the fixed scratch array on `device`, which must be the
// current device; looked up once per device.
hipError_t noalloc_scratch(int device, void** ptr);

hipError_t launch_prep(const PrepParams& P, hipStream_t s);
hipError_t launch_count(bool single_delim, const CountParams& P, int grid, hipStream_t s);
hipError_t launch_scan(const ScanParams& P, hipStream_t s);
hipError_t launch_parse(int k, bool single_delim, const ParseParams& P, int grid, hipStream_t s);
hipError_t launch_fallback(const FallbackParams& P, int grid, hipStream_t s);
hipError_t launch_reduce_final(const FallbackParams& P, hipStream_t s);

}  // namespace ffp
