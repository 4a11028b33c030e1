// Frozen-schedule advance that allocates nothing (swe_advance_dt_noalloc of
// include/swe.h), for callers that cannot allocate device memory.
//
// swe_advance_dt records the time steps it takes through a device buffer
// that the context allocates on demand (and grows with the step count).
// This variant stages them in `scratch`, a fixed array in the library's own
// device memory (one copy per GPU, kept until the process ends), so that a
// call on a context whose workspace is already in place calls no hipMalloc,
// hipFree or allocating library routine.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "swe.h"
#include "swe_ctx.hpp"

namespace {

// Most time steps one call may record (128 KiB of device memory per GPU).
constexpr int64_t kScratchSteps = SWE_NOALLOC_MAX_STEPS;

// Every call on a GPU shares this array: calls that overlap on one GPU
// (several contexts on different streams) race on it.
static __device__ __align__(256) __attribute__((used))
double scratch[kScratchSteps];

// Device address of `scratch` on each GPU, looked up once per device with
// that device current (the array's host-side name is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

swe_status scratch_address(swe_ctx *c, double **out)
{
    if (c->device >= kMaxDevices)
        return swe::ctx_fail(c, SWE_EDEVICE,
                             "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[c->device]) {
        hipError_t e = hipSetDevice(c->device);
        if (e == hipSuccess) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e == hipSuccess && p) g_scratch_ptr[c->device] = (double *)p;
        }
        if (e != hipSuccess || !g_scratch_ptr[c->device])
            return swe::ctx_fail(
                c, SWE_EDEVICE,
                std::string("address of the time-step scratch array: ") +
                    hipGetErrorString(e));
    }
    *out = g_scratch_ptr[c->device];
    return SWE_OK;
}

}  // namespace

extern "C" {

swe_status swe_advance_dt_noalloc(swe_ctx *c, int64_t n, const double *dt,
                                  double *dt_out)
{
    swe_status st = swe::ctx_advance_dt_check(c, n, dt);
    if (st != SWE_OK || n == 0) return st;
    if (dt_out && n > kScratchSteps)
        return swe::ctx_fail(
            c, SWE_EINVAL,
            "swe_advance_dt_noalloc records at most " +
                std::to_string(kScratchSteps) + " time steps per call (asked " +
                std::to_string(n) + "); split the run into several calls");
    // the device workspace must already be in place: bound by the caller,
    // or allocated by an earlier call
    if (!c->dev_ready && !c->ws)
        return swe::ctx_fail(
            c, SWE_ENOTREADY,
            "no device workspace yet: bind one with swe_bind_workspace, or "
            "let an earlier call (e.g. swe_advance of 0 steps) allocate it");
    double *log = nullptr;
    if (dt_out && (st = scratch_address(c, &log))) return st;
    if ((st = swe::ctx_prepare(c))) return st;
    return swe::ctx_advance_dt(c, n, dt, dt_out, log);
}

}  // extern "C"
