// Launcher of the per-tag discharge sums (swe_monitor.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace swe {

// out[2 t], out[2 t + 1] = the sums of rate and vol over tag t's boundary
// slots tag_slot[tag_ptr[t] .. tag_ptr[t + 1]), t < n_tags
hipError_t launch_discharge_tags(const double *rate, const double *vol,
                                 const int32_t *tag_ptr,
                                 const int32_t *tag_slot, int n_tags,
                                 double *out, hipStream_t s);

}  // namespace swe
