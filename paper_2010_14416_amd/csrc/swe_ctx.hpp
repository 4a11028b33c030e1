// Internal state of a context (struct swe_ctx of include/swe.h), shared by
// the C interface (swe_api.cpp) and the ensemble (swe_ensemble.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "swe.h"
#include "swe_device.hpp"
#include "swe_mesh.hpp"

namespace swe {

// Device buffers, carved from one workspace (256-byte aligned pieces).
struct DevBufs {
    double *h[2], *hu[2], *hv[2];
    double *z, *man, *gm2, *area, *inr;
    int32_t *internal_of_user, *user_of_internal;
    int32_t *blk_edge;
    int32_t *be_a, *be_b;
    double *be_nx, *be_ny, *be_len;
    BcEntry *bc;
    Clock *clock;
    double *ledger;
    int32_t *quiet;
    double *mon_rate, *mon_vol;   // per boundary slot
    int32_t *blk_bnd;             // per block, 4 values
    uint32_t *run;                // run marks, 2 x n_blocks
    unsigned long long *act;      // per block, a bit per cell (StepArgs)
    double *h_max, *t_wet;        // per cell (internal order)
    MonPtrs *mon;                 // the five monitor addresses above
    double *part_mass;
    unsigned long long *part_wet;
    unsigned *flag;
    // boundary slots per tag (tag_ptr: SWE_MAX_TAG + 1 offsets into
    // tag_slot, slots in increasing order) and the per-tag rate and volume
    // sums of an asynchronous discharge copy (2 x SWE_MAX_TAG)
    int32_t *tag_ptr, *tag_slot;
    double *tag_out;
};

constexpr int kDiagParts = 1024;

}  // namespace swe

struct swe_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    swe_params params{};
    std::string err;
    bool has_mesh = false;
    swe::BlockMesh mesh;
    std::vector<uint8_t> groups;   // cell groups for the next set_mesh
    int32_t wet_band = -1;         // >= 0: groups is a wet mask
    swe::MonPtrs mon_host{};       // source of the device copy d.mon
    // host copies in internal order; *_dirty: newer than the device copy
    std::vector<double> z, man, h, hu, hv;
    bool z_dirty = false, man_dirty = false, state_dirty = false;
    bool gm2_dirty = true;
    std::vector<swe::BcEntry> bc;        // per tag
    std::vector<swe::BcEntry> bc_slot;   // per boundary slot
    bool bc_dirty = true;
    // device
    bool dev_ready = false;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    swe::DevBufs d{};
    int cur_buf = 0;           // ping-pong buffer holding the current state
    int cur_slot = 0;          // clock slot read by the next step
    bool dt_valid = false;     // clock slot cur_slot holds min R/s of state
    bool clock_dirty = true;   // host t/step must be pushed to the device
    double t_host = 0.0;       // valid when t_known
    bool t_known = true;
    int64_t step_host = 0;
    double last_dt_host = 0.0;
    long long step_index = 0;  // steps launched since the mesh was set
    bool uploaded = false;     // host memory queued on the stream
    bool quiet_dirty = true;   // state buffers written outside a step
    bool mon_dirty = true;     // monitors to be reset before the next step
    double *dt_dev = nullptr;  // time-step schedule (library-allocated)
    int64_t dt_cap = 0;
    swe::StepGraph graph;      // captured step runs (graph_steps > 0)
    // asynchronous discharge copies: a stream of the library's own (default
    // priority), an event marking the step they follow, one marking the
    // copy's end
    hipStream_t side = nullptr;
    hipEvent_t ev_step = nullptr, ev_copy = nullptr;
    bool copy_pending = false;
    std::vector<int32_t> tag_ptr_host, tag_slot_host;   // upload sources
};

namespace swe {

// Internal steps shared by the C interface and the adjoint.
swe_status ctx_prepare(swe_ctx *c);
swe_status ctx_fail(swe_ctx *c, swe_status st, const std::string &msg);
swe_status ctx_read_clock(swe_ctx *c);
StepArgs ctx_step_args(swe_ctx *c, double t_end);
// Enqueues n steps; advances the buffers, clock slot and step index. With
// dt_fixed (host, n values) step k takes dt_fixed[k] as its time step;
// with dt_log (device, n values) the time step of step k is copied there.
// With slots, the steps run outside the ping-pong buffers: step k reads the
// state at slots + k * stride (h, hu, hv, n_cells values each) and writes
// every cell of slots + (k + 1) * stride. With run_log (device), step k
// records which blocks ran at run_log + k * n_blocks; with r_log (device),
// its summed edge contributions at r_log + k * 3 n_cells.
swe_status ctx_enqueue(swe_ctx *c, StepArgs &a, int64_t n,
                       const double *dt_fixed, double *dt_log,
                       double *slots = nullptr, size_t stride = 0,
                       uint8_t *run_log = nullptr, double *r_log = nullptr);
// One step from the state arrays `in` (h, hu, hv) into `out`, outside the
// context's ping-pong buffers, with time step dt (monitors not updated);
// with run_log (device, n_blocks values), which blocks ran; with r_out
// (device, 3 n_cells values), the summed edge contributions.
swe_status ctx_step_between(swe_ctx *c, const double *const in[3],
                            double *const out[3], double dt,
                            uint8_t *run_log = nullptr,
                            double *r_out = nullptr);
// Argument checks of a frozen-schedule advance (no device use).
swe_status ctx_advance_dt_check(swe_ctx *c, int64_t n, const double *dt);
// n steps with the host time steps dt (or the CFL time steps when dt is
// null) on a prepared context; with dt_out, the time steps taken go through
// the device buffer `log` (n values) to the host array dt_out. Synchronises.
swe_status ctx_advance_dt(swe_ctx *c, int64_t n, const double *dt,
                          double *dt_out, double *log);
// Device buffer of at least n time steps in c->dt_dev.
swe_status ctx_dt_buffer(swe_ctx *c, int64_t n);

}  // namespace swe

