// Device arguments and launchers of the discrete adjoint of one step
// (swe_adjoint.hip), driven by swe_adjoint.cpp.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "swe_device.hpp"

namespace swe {

struct AdjArgs {
    // mesh (internal order), as for the step
    const int32_t *blk_edge;
    const int32_t *be_a;
    const int32_t *be_b;
    const double *be_nx;
    const double *be_ny;
    const double *be_len;
    const double *z;
    const double *gm2;
    const double *area;
    const BcEntry *bc;
    // U^k, the state the step starts from
    const double *h;
    const double *hu;
    const double *hv;
    // lambda^{k+1} in, lambda^k out
    const double *lam_h;
    const double *lam_hu;
    const double *lam_hv;
    double *lam_out_h;
    double *lam_out_hu;
    double *lam_out_hv;
    // per cell: direct part of lambda^k and the adjoint of the summed
    // contribution R (written by the cell pass, read by the edge pass)
    double *ld_h;
    double *ld_hu;
    double *ld_hv;
    double *lr_h;
    double *lr_hu;
    double *lr_hv;
    // gradients, accumulated over the reverse steps
    double *grad_gm2;
    double *grad_z;
    // null, or per block 0 if the block was dormant in the forward step
    // (its cells kept their quiet dry state: lambda_h passes through,
    // lambda_hu and lambda_hv become 0, no gradient), else 1
    const uint8_t *ran;
    // null, or the summed edge contributions R of the forward step (3 x
    // n_cells, stored by it): the cell pass then reads R instead of
    // evaluating the block's edges again
    const double *R;
    double g, h_dry, dt;
    int32_t n_cells;
    int32_t n_blocks;
};

// One reverse step (cell pass, then edge pass); blocks of 256 cells.
hipError_t launch_adjoint_step(const AdjArgs &a, int block_cells,
                               hipStream_t s);
// out = gm2_grad * 2 g m (the Manning gradient from that of g m^2).
hipError_t launch_manning_gradient(const double *gm2_grad, const double *man,
                                   double g, int64_t n, double *out,
                                   hipStream_t s);

}  // namespace swe
