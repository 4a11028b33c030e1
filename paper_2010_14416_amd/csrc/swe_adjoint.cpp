// Gradient of a gauge misfit by the discrete adjoint (swe_adjoint_gauges of
// include/swe.h), for inverse analysis: which Manning field and bed make
// the model match observed depths.
//
// Forward: `steps` ordinary steps from the context's state, recording each
// time step, with the state saved every K steps (K = checkpoint interval).
// Reverse: segment by segment from the last, the state is restored from its
// checkpoint and the segment replayed with its recorded time steps (bit for
// bit the forward states) straight into the segment's state slots; then the
// adjoint steps run backwards through them. Memory: about K + ceil(steps / K)
// states of 24 B per cell. K = 1 keeps every state: the forward steps write
// straight into their slots and nothing is replayed. Unless the caller fixes
// K, it is the smallest interval whose states fit in half the free device
// memory (a mesh of a million cells keeps thousands of states in HBM), and at
// most ceil(sqrt(steps)), which minimises the memory.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "swe.h"
#include "swe_adjoint.hpp"
#include "swe_ctx.hpp"
#include "swe_device.hpp"

using swe::ctx_fail;

namespace {

#define ADJCHK(ctx, call)                                                  \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess)                                              \
            return ctx_fail(ctx, SWE_EDEVICE, std::string(#call) + ": " +  \
                                                  hipGetErrorString(e_));  \
    } while (0)

struct DeviceScratch {
    void *p = nullptr;
    ~DeviceScratch()
    {
        if (p) (void)hipFree(p);
    }
};

// Copies the three state arrays of the context's current buffer to dst
// (h, hu, hv, n values each) or back.
swe_status copy_state(swe_ctx *c, double *dst, bool to_ctx)
{
    const size_t n = size_t(c->mesh.n_cells);
    const int b = c->cur_buf;
    double *s[3] = {c->d.h[b], c->d.hu[b], c->d.hv[b]};
    for (int k = 0; k < 3; ++k) {
        double *x = dst + k * n;
        ADJCHK(c, hipMemcpyAsync(to_ctx ? s[k] : x, to_ctx ? x : s[k], n * 8,
                                 hipMemcpyDeviceToDevice, c->stream));
    }
    return SWE_OK;
}

// Arrays of 3 n_cells values held for interval K: every state and the
// summed edge contributions R of every step when K = 1; else the
// checkpoints, the slots of one segment, the final state and the R of the
// replayed steps of a segment.
int64_t states_held(int64_t steps, int64_t K)
{
    return K == 1 ? 2 * steps + 1 : (steps + K - 1) / K + K + 1 + (K - 1);
}

int64_t pick_interval(int64_t steps, size_t state_bytes, size_t other_bytes)
{
    const int64_t k_min_memory =
        std::max<int64_t>(1, int64_t(std::ceil(std::sqrt(double(steps)))));
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return k_min_memory;
    const double budget = 0.5 * double(free_b) - double(other_bytes);
    for (int64_t K = 1; K < k_min_memory; ++K)
        if (double(states_held(steps, K)) * double(state_bytes) <= budget)
            return K;
    return k_min_memory;
}

}  // namespace

extern "C" swe_status swe_adjoint_gauges(swe_ctx *c, int64_t steps,
                                         int32_t n_gauges,
                                         const int32_t *gauges,
                                         const double *h_target,
                                         int32_t checkpoint_every,
                                         double *loss, double *grad_manning,
                                         double *grad_z)
{
    if (!c) return SWE_EINVAL;
    if (!c->has_mesh) return ctx_fail(c, SWE_ENOTREADY, "no mesh set");
    if (steps < 1) return ctx_fail(c, SWE_EINVAL, "need at least one step");
    if (n_gauges < 1 || !gauges || !h_target || !loss)
        return ctx_fail(c, SWE_EINVAL, "need gauges, targets and a loss");
    const int64_t nc = c->mesh.n_cells;
    for (int32_t k = 0; k < n_gauges; ++k)
        if (gauges[k] < 0 || gauges[k] >= nc || !std::isfinite(h_target[k]))
            return ctx_fail(c, SWE_EINVAL,
                            "gauge " + std::to_string(k) +
                                " out of range or with a non-finite target");
    if (c->mesh.block_cells != 256)
        return ctx_fail(c, SWE_EINVAL, "the adjoint needs block_cells = 256");
    if (checkpoint_every < 0)
        return ctx_fail(c, SWE_EINVAL, "negative checkpoint interval");
    swe_status st = swe::ctx_prepare(c);
    if (st) return st;
    if (!c->t_known && (st = swe::ctx_read_clock(c))) return st;

    const size_t n = size_t(nc), nb = size_t(c->mesh.n_blocks);
    const size_t n_state = 3 * n;
    // besides the states: adjoints, gradients, ledger copy
    const size_t other = 2 * n_state + 2 * n_state + 3 * n + nb;
    const int64_t K = checkpoint_every > 0
                          ? std::min<int64_t>(checkpoint_every, steps)
                          : pick_interval(steps, n_state * 8, other * 8);
    const int64_t nseg = (steps + K - 1) / K;
    // which blocks ran in each forward step (K = 1) or replayed step
    const size_t log_bytes = size_t(K == 1 ? steps : K) * nb;
    const size_t doubles = size_t(states_held(steps, K)) * n_state + other +
                           (log_bytes + 7) / 8;
    DeviceScratch scratch;
    {
        hipError_t e = hipMalloc(&scratch.p, doubles * 8);
        if (e != hipSuccess)
            return ctx_fail(c, SWE_ENOMEM,
                            "adjoint scratch of " +
                                std::to_string(doubles * 8) +
                                " bytes: " + hipGetErrorString(e));
    }
    double *p = (double *)scratch.p;
    // with K = 1, ckpt holds the state before every step and final_state,
    // right behind it, is the slot the last step writes
    double *ckpt = p;                    p += size_t(nseg) * n_state;
    double *seg = p;                     p += K > 1 ? size_t(K) * n_state : 0;
    double *final_state = p;             p += n_state;
    // the summed edge contributions of every step (K = 1) or of the
    // replayed steps of a segment
    double *r_log = p;   p += size_t(K == 1 ? steps : K - 1) * n_state;
    double *lam[2] = {p, p + n_state};   p += 2 * n_state;
    double *ld = p;                      p += n_state;
    double *lr = p;                      p += n_state;
    double *g_gm2 = p;                   p += n;
    double *g_z = p;                     p += n;
    double *g_m = p;                     p += n;
    double *ledger_copy = p;             p += nb;
    uint8_t *run_log = (uint8_t *)p;

    // forward: ordinary steps, time steps recorded, checkpoints
    if ((st = swe::ctx_dt_buffer(c, steps))) return st;
    if (K == 1) {
        if ((st = copy_state(c, ckpt, false))) return st;
        swe::StepArgs a = swe::ctx_step_args(c, INFINITY);
        if ((st = swe::ctx_enqueue(c, a, steps, nullptr, c->dt_dev, ckpt,
                                   n_state, run_log, r_log)))
            return st;
    } else {
        for (int64_t s = 0; s < nseg; ++s) {
            const int64_t m = std::min(K, steps - s * K);
            if ((st = copy_state(c, ckpt + size_t(s) * n_state, false)))
                return st;
            swe::StepArgs a = swe::ctx_step_args(c, INFINITY);
            if ((st = swe::ctx_enqueue(c, a, m, nullptr, c->dt_dev + s * K)))
                return st;
        }
        if ((st = copy_state(c, final_state, false))) return st;
    }
    std::vector<double> dts(static_cast<size_t>(steps));
    ADJCHK(c, hipMemcpyAsync(dts.data(), c->dt_dev, size_t(steps) * 8,
                             hipMemcpyDeviceToHost, c->stream));
    if ((st = swe::ctx_read_clock(c))) return st;   // also checks health
    const double t_final = c->t_host;
    const int64_t steps_final = c->step_host;
    ADJCHK(c, hipMemcpyAsync(ledger_copy, c->d.ledger, nb * 8,
                             hipMemcpyDeviceToDevice, c->stream));

    // loss and lambda^N = dL/dU^N
    std::vector<double> hN(n), lam_h(n, 0.0);
    ADJCHK(c, hipMemcpyAsync(hN.data(), final_state, n * 8,
                             hipMemcpyDeviceToHost, c->stream));
    ADJCHK(c, hipStreamSynchronize(c->stream));
    double L = 0.0;
    for (int32_t k = 0; k < n_gauges; ++k) {
        const int32_t i = c->mesh.internal_of_user[gauges[k]];
        const double r = hN[i] - h_target[k];
        L += r * r;
        lam_h[i] += 2.0 * r;
    }
    *loss = L;
    double *lam_cur = lam[0], *lam_next = lam[1];
    ADJCHK(c, hipMemcpyAsync(lam_cur, lam_h.data(), n * 8,
                             hipMemcpyHostToDevice, c->stream));
    ADJCHK(c, swe::launch_fill_f64(lam_cur + n, 0.0, int64_t(2 * n),
                                   c->stream));
    ADJCHK(c, swe::launch_fill_f64(g_gm2, 0.0, int64_t(n), c->stream));
    ADJCHK(c, swe::launch_fill_f64(g_z, 0.0, int64_t(n), c->stream));

    swe::AdjArgs A{};
    A.blk_edge = c->d.blk_edge;
    A.be_a = c->d.be_a;
    A.be_b = c->d.be_b;
    A.be_nx = c->d.be_nx;
    A.be_ny = c->d.be_ny;
    A.be_len = c->d.be_len;
    A.z = c->d.z;
    A.gm2 = c->d.gm2;
    A.area = c->d.area;
    A.bc = c->d.bc;
    A.ld_h = ld;
    A.ld_hu = ld + n;
    A.ld_hv = ld + 2 * n;
    A.lr_h = lr;
    A.lr_hu = lr + n;
    A.lr_hv = lr + 2 * n;
    A.grad_gm2 = g_gm2;
    A.grad_z = g_z;
    A.g = c->params.g;
    A.h_dry = c->params.h_dry;
    A.n_cells = int32_t(nc);
    A.n_blocks = c->mesh.n_blocks;

    // reverse, segment by segment: replay the segment from its checkpoint
    // straight into the segment's state slots (slot 0 is the checkpoint),
    // then run its reverse steps backwards
    auto state_at = [&](int64_t s, int64_t j) {
        return j == 0 ? ckpt + size_t(s) * n_state : seg + size_t(j) * n_state;
    };
    for (int64_t s = nseg - 1; s >= 0; --s) {
        const int64_t m = std::min(K, steps - s * K);
        if (m > 1) {
            // the quiet counters and run marks describe the state the
            // context last stepped, not this checkpoint: every block runs
            // the replay's first two steps, dormant blocks only after that
            ADJCHK(c, swe::launch_fill_u32((unsigned *)c->d.quiet, 0u,
                                           int64_t(nb), c->stream));
            ADJCHK(c, swe::launch_fill_u32(c->d.run, 1u, 2 * int64_t(nb),
                                           c->stream));
        }
        for (int64_t j = 0; j + 1 < m; ++j) {
            const double *u = state_at(s, j);
            double *w = state_at(s, j + 1);
            const double *in[3] = {u, u + n, u + 2 * n};
            double *const out[3] = {w, w + n, w + 2 * n};
            if ((st = swe::ctx_step_between(c, in, out,
                                            dts[size_t(s * K + j)],
                                            run_log + size_t(j) * nb,
                                            r_log + size_t(j) * n_state)))
                return st;
        }
        for (int64_t j = m - 1; j >= 0; --j) {
            const double *u = state_at(s, j);
            A.h = u;
            A.hu = u + n;
            A.hv = u + 2 * n;
            A.lam_h = lam_cur;
            A.lam_hu = lam_cur + n;
            A.lam_hv = lam_cur + 2 * n;
            A.lam_out_h = lam_next;
            A.lam_out_hu = lam_next + n;
            A.lam_out_hv = lam_next + 2 * n;
            A.dt = dts[size_t(s * K + j)];
            // blocks dormant in the forward step (recorded by the forward
            // for K = 1, by the replay for the others; the segment's last
            // step was not replayed)
            A.ran = K == 1 ? run_log + size_t(s) * nb
                           : (j + 1 < m ? run_log + size_t(j) * nb : nullptr);
            A.R = K == 1 ? r_log + size_t(s) * n_state
                         : (j + 1 < m ? r_log + size_t(j) * n_state : nullptr);
            ADJCHK(c, swe::launch_adjoint_step(A, 256, c->stream));
            std::swap(lam_cur, lam_next);
        }
    }

    // gradients in user order
    ADJCHK(c, swe::launch_manning_gradient(g_gm2, c->d.man, c->params.g,
                                           int64_t(nc), g_m, c->stream));
    std::vector<double> gm(n), gz(n);
    ADJCHK(c, hipMemcpyAsync(gm.data(), g_m, n * 8, hipMemcpyDeviceToHost,
                             c->stream));
    ADJCHK(c, hipMemcpyAsync(gz.data(), g_z, n * 8, hipMemcpyDeviceToHost,
                             c->stream));
    // the context ends at the forward's final state, time and ledger
    if ((st = copy_state(c, final_state, true))) return st;
    ADJCHK(c, swe::launch_fill_u32((unsigned *)c->d.quiet, 0u, int64_t(nb),
                                   c->stream));
    ADJCHK(c, swe::launch_fill_u32(c->d.run, 1u, 2 * int64_t(nb), c->stream));
    ADJCHK(c, hipMemcpyAsync(c->d.ledger, ledger_copy, nb * 8,
                             hipMemcpyDeviceToDevice, c->stream));
    ADJCHK(c, swe::launch_clock_set(c->d.clock, t_final, steps_final,
                                    c->step_index, c->stream));
    ADJCHK(c, hipStreamSynchronize(c->stream));
    c->t_host = t_final;
    c->step_host = steps_final;
    c->t_known = true;
    c->dt_valid = false;
    c->mon_dirty = true;
    for (int64_t u = 0; u < nc; ++u) {
        const int32_t i = c->mesh.internal_of_user[u];
        if (grad_manning) grad_manning[u] = gm[i];
        if (grad_z) grad_z[u] = gz[i];
    }
    return swe::ctx_prepare(c);
}
