// Per-tag sums of the discharge monitors for their asynchronous copy to the
// host (swe_discharge_async of include/swe.h; the rates of sec. 5.3.2).
#include <hip/hip_runtime.h>

#include "swe_monitor.hpp"

namespace swe {
namespace {

// Thread t adds the rate and volume of tag t's boundary slots in increasing
// slot order (the order of the host-side sums of swe_get_discharge, so the
// same bits).
__global__ __launch_bounds__(256) void discharge_tags_kernel(
    const double *rate, const double *vol, const int32_t *tag_ptr,
    const int32_t *tag_slot, int n_tags, double *out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tags) return;
    double r = 0.0, v = 0.0;
    for (int k = tag_ptr[t]; k < tag_ptr[t + 1]; ++k) {
        r += rate[tag_slot[k]];
        v += vol[tag_slot[k]];
    }
    out[2 * t] = r;
    out[2 * t + 1] = v;
}

}  // namespace

hipError_t launch_discharge_tags(const double *rate, const double *vol,
                                 const int32_t *tag_ptr,
                                 const int32_t *tag_slot, int n_tags,
                                 double *out, hipStream_t s)
{
    hipLaunchKernelGGL(discharge_tags_kernel, dim3((n_tags + 255) / 256),
                       dim3(256), 0, s, rate, vol, tag_ptr, tag_slot, n_tags,
                       out);
    return hipGetLastError();
}

}  // namespace swe
