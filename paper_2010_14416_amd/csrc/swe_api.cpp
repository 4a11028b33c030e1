// C interface (include/swe.h) of the shallow-water step: context, input
// validation and reordering on the host, device memory, the step loop.
#include "swe.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "swe_ctx.hpp"
#include "swe_device.hpp"
#include "swe_mesh.hpp"
#include "swe_monitor.hpp"

using swe::BcEntry;
using swe::BlockMesh;
using swe::Clock;
using swe::DevBufs;
using swe::kDiagParts;

namespace {

thread_local std::string g_create_error;

swe_status fail(swe_ctx *c, swe_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

swe_status hip_fail(swe_ctx *c, hipError_t e, const char *what)
{
    return fail(c, SWE_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, call)                                                  \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);           \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace layout: returns the total size; fills d when base != nullptr.
size_t layout(const BlockMesh &m, char *base, DevBufs *d)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const size_t nc = size_t(m.n_cells), nb = size_t(m.n_blocks);
    const size_t nbe = m.be_a.size();
    DevBufs t{};
    for (int k = 0; k < 2; ++k) {
        t.h[k] = (double *)take(nc * 8);
        t.hu[k] = (double *)take(nc * 8);
        t.hv[k] = (double *)take(nc * 8);
    }
    t.z = (double *)take(nc * 8);
    t.man = (double *)take(nc * 8);
    t.gm2 = (double *)take(nc * 8);
    t.area = (double *)take(nc * 8);
    t.inr = (double *)take(nc * 8);
    t.internal_of_user = (int32_t *)take(nc * 4);
    t.user_of_internal = (int32_t *)take(nc * 4);
    t.blk_edge = (int32_t *)take((nb + 1) * 4);
    t.be_a = (int32_t *)take(nbe * 4);
    t.be_b = (int32_t *)take(nbe * 4);
    t.be_nx = (double *)take(nbe * 8);
    t.be_ny = (double *)take(nbe * 8);
    t.be_len = (double *)take(nbe * 8);
    const size_t nbnd = m.bnd_tag.size() > 0 ? m.bnd_tag.size() : 1;
    t.bc = (BcEntry *)take(sizeof(BcEntry) * nbnd);
    t.clock = (Clock *)take(sizeof(Clock));
    t.ledger = (double *)take(nb * 8);
    t.quiet = (int32_t *)take(nb * 4);
    t.mon_rate = (double *)take(nbnd * 8);
    t.mon_vol = (double *)take(nbnd * 8);
    t.blk_bnd = (int32_t *)take(nb * 16);
    t.act = (unsigned long long *)take(nb * (m.block_cells / 64) * 8);
    t.run = (uint32_t *)take(2 * nb * 4);
    t.h_max = (double *)take(nc * 8);
    t.t_wet = (double *)take(nc * 8);
    t.mon = (swe::MonPtrs *)take(sizeof(swe::MonPtrs));
    t.part_mass = (double *)take(kDiagParts * 8);
    t.part_wet = (unsigned long long *)take(kDiagParts * 8);
    t.flag = (unsigned *)take(256);
    t.tag_ptr = (int32_t *)take((SWE_MAX_TAG + 1) * 4);
    t.tag_slot = (int32_t *)take(nbnd * 4);
    t.tag_out = (double *)take(2 * SWE_MAX_TAG * 8);
    if (d) *d = t;
    return off;
}

bool valid_block_cells(int32_t b)
{
    return b == 64 || b == 128 || b == 256 || b == 512;
}

swe_status require_mesh(swe_ctx *c)
{
    if (!c) return SWE_EINVAL;
    if (!c->has_mesh) return fail(c, SWE_ENOTREADY, "no mesh set");
    return SWE_OK;
}

template <typename T>
swe_status upload(swe_ctx *c, T *dst, const T *src, size_t n)
{
    if (n == 0) return SWE_OK;
    HIPCHK(c, hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice,
                             c->stream));
    c->uploaded = true;
    return SWE_OK;
}

swe_status read_clock(swe_ctx *c, Clock *out);

// Allocates (or adopts) the workspace and uploads whatever the host holds
// newer than the device.
swe_status prepare(swe_ctx *c)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    HIPCHK(c, hipSetDevice(c->device));
    const BlockMesh &m = c->mesh;
    const size_t nc = size_t(m.n_cells);
    if (!c->dev_ready) {
        const size_t need = layout(m, nullptr, nullptr);
        if (!c->ws) {
            void *p = nullptr;
            hipError_t e = hipMalloc(&p, need);
            if (e != hipSuccess)
                return fail(c, SWE_ENOMEM,
                            std::string("device allocation of ") +
                                std::to_string(need) + " bytes failed: " +
                                hipGetErrorString(e));
            c->ws = p;
            c->ws_bytes = need;
            c->ws_owned = true;
        }
        layout(m, (char *)c->ws, &c->d);
        DevBufs &d = c->d;
        if ((st = upload(c, d.area, m.area.data(), nc))) return st;
        if ((st = upload(c, d.inr, m.inradius.data(), nc))) return st;
        if ((st = upload(c, d.internal_of_user, m.internal_of_user.data(), nc)))
            return st;
        if ((st = upload(c, d.user_of_internal, m.user_of_internal.data(), nc)))
            return st;
        if ((st = upload(c, d.blk_edge, m.blk_edge.data(), m.blk_edge.size())))
            return st;
        if ((st = upload(c, d.blk_bnd, m.blk_bnd.data(), m.blk_bnd.size())))
            return st;
        {
            // boundary slots of each tag, in increasing slot order
            const std::vector<int32_t> &bt = m.bnd_tag;
            std::vector<int32_t> ptr(SWE_MAX_TAG + 1, 0), slot(bt.size());
            for (int32_t t : bt) ++ptr[size_t(t) + 1];
            for (int k = 0; k < SWE_MAX_TAG; ++k) ptr[k + 1] += ptr[k];
            std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
            for (size_t k = 0; k < bt.size(); ++k)
                slot[size_t(fill[size_t(bt[k])]++)] = int32_t(k);
            c->tag_ptr_host = ptr;
            c->tag_slot_host = slot;
            if ((st = upload(c, d.tag_ptr, c->tag_ptr_host.data(),
                             c->tag_ptr_host.size())))
                return st;
            if (!slot.empty() &&
                (st = upload(c, d.tag_slot, c->tag_slot_host.data(),
                             slot.size())))
                return st;
        }
        c->mon_host = swe::MonPtrs{d.mon_rate, d.mon_vol, d.blk_bnd, d.h_max,
                              d.t_wet};
        if ((st = upload(c, d.mon, &c->mon_host, 1))) return st;
        const size_t nbe = m.be_a.size();
        if ((st = upload(c, d.be_a, m.be_a.data(), nbe))) return st;
        if ((st = upload(c, d.be_b, m.be_b.data(), nbe))) return st;
        if ((st = upload(c, d.be_nx, m.be_nx.data(), nbe))) return st;
        if ((st = upload(c, d.be_ny, m.be_ny.data(), nbe))) return st;
        if ((st = upload(c, d.be_len, m.be_len.data(), nbe))) return st;
        HIPCHK(c, swe::launch_fill_f64(d.ledger, 0.0, m.n_blocks, c->stream));
        c->dev_ready = true;
        c->z_dirty = c->man_dirty = c->state_dirty = true;
        c->bc_dirty = c->gm2_dirty = c->clock_dirty = true;
        c->dt_valid = false;
        c->cur_buf = 0;
        c->cur_slot = 0;
    }
    DevBufs &d = c->d;
    // any input of the step changed: no block may be taken as dormant
    if (c->z_dirty || c->man_dirty || c->gm2_dirty || c->bc_dirty)
        c->quiet_dirty = true;
    if (c->z_dirty) {
        if ((st = upload(c, d.z, c->z.data(), nc))) return st;
        c->z_dirty = false;
    }
    if (c->man_dirty) {
        if ((st = upload(c, d.man, c->man.data(), nc))) return st;
        c->man_dirty = false;
        c->gm2_dirty = true;
    }
    if (c->gm2_dirty) {
        HIPCHK(c, swe::launch_gm2(d.man, d.gm2, nc, c->params.g, c->stream));
        c->gm2_dirty = false;
    }
    if (c->state_dirty) {
        if ((st = upload(c, d.h[c->cur_buf], c->h.data(), nc))) return st;
        if ((st = upload(c, d.hu[c->cur_buf], c->hu.data(), nc))) return st;
        if ((st = upload(c, d.hv[c->cur_buf], c->hv.data(), nc))) return st;
        c->state_dirty = false;
        c->dt_valid = false;
        c->quiet_dirty = true;
        c->mon_dirty = true;
    }
    if (c->quiet_dirty) {
        // the step kernel may skip stores, and dormant blocks, only after
        // two steps from here
        HIPCHK(c, swe::launch_fill_u32((unsigned *)d.quiet, 0u, m.n_blocks,
                                       c->stream));
        HIPCHK(c, swe::launch_fill_u32(d.run, 1u, 2 * int64_t(m.n_blocks),
                                       c->stream));
        HIPCHK(c, swe::launch_fill_u32((unsigned *)d.act, 0u,
                                       int64_t(m.n_blocks) * m.block_cells / 32,
                                       c->stream));
        c->quiet_dirty = false;
    }
    if (c->bc_dirty) {
        // inflow discharge per unit length of each tag, then one entry per
        // boundary slot
        for (int k = 0; k < SWE_MAX_TAG; ++k) {
            BcEntry &b = c->bc[k];
            const double L = c->mesh.tag_length[k];
            b.q = (b.kind == SWE_BC_INFLOW && L > 0.0) ? b.value / L : 0.0;
        }
        const std::vector<int32_t> &bt = c->mesh.bnd_tag;
        c->bc_slot.resize(bt.size());
        for (size_t k = 0; k < bt.size(); ++k) c->bc_slot[k] = c->bc[bt[k]];
        if ((st = upload(c, d.bc, c->bc_slot.data(), bt.size()))) return st;
        c->bc_dirty = false;
    }
    if (c->clock_dirty) {
        HIPCHK(c, swe::launch_clock_set(d.clock, c->t_host, c->step_host,
                                        c->step_index,
                                        c->stream));
        c->clock_dirty = false;
        c->dt_valid = false;
    }
    if (c->params.monitors && c->mon_dirty) {
        if (!c->t_known) {
            Clock ck;
            if ((st = read_clock(c, &ck))) return st;
        }
        const size_t nbnd = c->mesh.bnd_tag.size();
        HIPCHK(c, swe::launch_fill_f64(d.mon_rate, 0.0, nbnd, c->stream));
        HIPCHK(c, swe::launch_fill_f64(d.mon_vol, 0.0, nbnd, c->stream));
        HIPCHK(c, swe::launch_envelope_reset(d.h[c->cur_buf], nc,
                                             c->params.h_dry, c->t_host,
                                             d.h_max, d.t_wet, c->stream));
        c->mon_dirty = false;
    }
    if (!c->dt_valid) {
        // min over wet cells of R_i / s_i of the current state, into the
        // slot the next step reads
        HIPCHK(c, swe::launch_slot_reset(d.clock, c->cur_slot, c->stream));
        HIPCHK(c, swe::launch_min_rs(d.h[c->cur_buf], d.hu[c->cur_buf],
                                     d.hv[c->cur_buf], d.inr, nc,
                                     c->params.g, c->params.h_dry, d.clock,
                                     c->cur_slot, c->stream));
        c->dt_valid = true;
    }
    // host arrays were handed to the stream: wait before returning so the
    // caller may free or reuse its inputs
    if (c->uploaded) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->uploaded = false;
    }
    return SWE_OK;
}

swe_status read_clock(swe_ctx *c, Clock *out)
{
    HIPCHK(c, hipMemcpyAsync(out, c->d.clock, sizeof(Clock),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->t_host = out->t[c->cur_slot];
    c->t_known = true;
    c->step_host = out->steps;
    c->last_dt_host = out->last_dt;
    if (out->health) {
        std::string why = (out->health & 1u) ? "non-finite state"
                                             : "unbounded time step (no wet "
                                               "cell, dt_max and t_end "
                                               "infinite)";
        return fail(c, SWE_ENUMERIC,
                    why + " at step " + std::to_string(out->bad_step));
    }
    return SWE_OK;
}

// Reads the device clock (synchronising the stream) and reports a step
// that raised its health word since the clock was last set: the results a
// caller reads after such a step are not those of a valid run.
swe_status check_health(swe_ctx *c)
{
    Clock ck;
    return read_clock(c, &ck);
}

swe_status check_flag(swe_ctx *c, bool *bad)
{
    unsigned f = 0;
    HIPCHK(c, hipMemcpyAsync(&f, c->d.flag, sizeof f, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *bad = f != 0;
    return SWE_OK;
}

enum class Field { z, manning };

// Cell field given by the caller (user order) into the internal host copy,
// or (device memory) straight into the device array.
swe_status set_field(swe_ctx *c, const double *src, swe_mem mem, Field f)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    const bool nonneg = f == Field::manning;
    const char *name = f == Field::z ? "bathymetry" : "manning";
    std::vector<double> &host = f == Field::z ? c->z : c->man;
    bool &dirty = f == Field::z ? c->z_dirty : c->man_dirty;
    if (!src) return fail(c, SWE_EINVAL, std::string(name) + " is NULL");
    const int64_t nc = c->mesh.n_cells;
    if (mem == SWE_MEM_HOST) {
        for (int64_t u = 0; u < nc; ++u)
            if (!std::isfinite(src[u]) || (nonneg && !(src[u] >= 0.0)))
                return fail(c, SWE_ESTATE,
                            std::string(name) + " invalid at cell " +
                                std::to_string(u));
        for (int64_t i = 0; i < nc; ++i)
            host[i] = src[c->mesh.user_of_internal[i]];
        dirty = true;
        if (f == Field::manning) c->gm2_dirty = true;
        return SWE_OK;
    }
    if (mem != SWE_MEM_DEVICE) return fail(c, SWE_EINVAL, "bad memory kind");
    if ((st = prepare(c))) return st;
    double *dev = f == Field::z ? c->d.z : c->d.man;
    HIPCHK(c, swe::launch_fill_u32(c->d.flag, 0u, 1, c->stream));
    HIPCHK(c, swe::launch_check_field(src, nc, nonneg ? 1 : 0, c->d.flag,
                                      c->stream));
    bool bad = false;
    if ((st = check_flag(c, &bad))) return st;
    if (bad) return fail(c, SWE_ESTATE, std::string(name) + " invalid");
    HIPCHK(c, swe::launch_gather1(src, dev, c->d.user_of_internal, nc,
                                  c->stream));
    if (f == Field::manning)
        HIPCHK(c, swe::launch_gm2(c->d.man, c->d.gm2, nc, c->params.g,
                                  c->stream));
    // an input of the step changed: no block may be taken as dormant (a
    // lowered bed under a fixed stage, say, must start inflow)
    c->quiet_dirty = true;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return prepare(c);
}

}  // namespace

extern "C" {

int swe_abi_version(void) { return SWE_ABI_VERSION; }

swe_status swe_default_params(swe_params *p)
{
    if (!p) return SWE_EINVAL;
    p->g = 9.81;
    p->cfl = 0.9;
    p->h_dry = 1e-6;
    p->dt_max = INFINITY;
    p->check_every = 64;
    p->block_cells = 256;
    p->reorder = 1;
    p->block_threads = 0;
    p->load_schedule = 0;
    p->monitors = 0;
    p->store_all = 0;
    p->graph_steps = 0;
    return SWE_OK;
}

swe_status swe_create(swe_ctx **out, int device)
{
    if (!out) return SWE_EINVAL;
    *out = nullptr;
    if (device < 0) {
        g_create_error = "negative device ordinal";
        return SWE_EINVAL;
    }
    swe_ctx *c = new (std::nothrow) swe_ctx();
    if (!c) {
        g_create_error = "out of memory";
        return SWE_ENOMEM;
    }
    c->device = device;
    swe_default_params(&c->params);
    c->bc.assign(SWE_MAX_TAG, BcEntry{SWE_BC_WALL, 0, 0.0, 0.0});
    *out = c;
    return SWE_OK;
}

void swe_destroy(swe_ctx *c)
{
    if (!c) return;
    if (c->side) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->side);
        (void)hipEventDestroy(c->ev_step);
        (void)hipEventDestroy(c->ev_copy);
        (void)hipStreamDestroy(c->side);
    }
    if ((c->ws_owned && c->ws) || c->dt_dev) {
        (void)hipSetDevice(c->device);
        if (c->ws_owned && c->ws) (void)hipFree(c->ws);
        if (c->dt_dev) (void)hipFree(c->dt_dev);
    }
    delete c;
}

const char *swe_last_error(const swe_ctx *c)
{
    return c ? c->err.c_str() : g_create_error.c_str();
}

swe_status swe_set_stream(swe_ctx *c, void *stream)
{
    if (!c) return SWE_EINVAL;
    c->stream = (hipStream_t)stream;
    return SWE_OK;
}

swe_status swe_set_params(swe_ctx *c, const swe_params *p)
{
    if (!c || !p) return SWE_EINVAL;
    if (!(p->g > 0.0) || !std::isfinite(p->g))
        return fail(c, SWE_EINVAL, "g must be positive and finite");
    if (!(p->cfl > 0.0) || !std::isfinite(p->cfl))
        return fail(c, SWE_EINVAL, "cfl must be positive and finite");
    if (!(p->h_dry >= 0.0) || !std::isfinite(p->h_dry))
        return fail(c, SWE_EINVAL, "h_dry must be >= 0 and finite");
    if (!(p->dt_max > 0.0))
        return fail(c, SWE_EINVAL, "dt_max must be positive");
    if (p->check_every < 1)
        return fail(c, SWE_EINVAL, "check_every must be >= 1");
    if (!valid_block_cells(p->block_cells))
        return fail(c, SWE_EINVAL, "block_cells must be 64, 128, 256 or 512");
    if (p->reorder != 0 && p->reorder != 1)
        return fail(c, SWE_EINVAL, "reorder must be 0 or 1");
    if (p->block_threads != 0 && p->block_threads != p->block_cells &&
        p->block_threads != 2 * p->block_cells)
        return fail(c, SWE_EINVAL,
                    "block_threads must be 0, block_cells or 2*block_cells");
    if (p->load_schedule != 0 && p->load_schedule != 1)
        return fail(c, SWE_EINVAL, "load_schedule must be 0 or 1");
    if (p->monitors != 0 && p->monitors != 1)
        return fail(c, SWE_EINVAL, "monitors must be 0 or 1");
    if (p->store_all != 0 && p->store_all != 1)
        return fail(c, SWE_EINVAL, "store_all must be 0 or 1");
    if (p->graph_steps < 0 || p->graph_steps > 4096 || p->graph_steps % 6)
        return fail(c, SWE_EINVAL,
                    "graph_steps must be 0 or a multiple of 6 up to 4096");
    const bool g_changed = p->g != c->params.g;
    const bool dt_changed = g_changed || p->h_dry != c->params.h_dry;
    if (p->monitors && !c->params.monitors) c->mon_dirty = true;
    c->params = *p;
    if (g_changed) c->gm2_dirty = true;
    if (dt_changed) {
        c->dt_valid = false;
        c->quiet_dirty = true;
    }
    return SWE_OK;
}

swe_status swe_get_params(const swe_ctx *c, swe_params *p)
{
    if (!c || !p) return SWE_EINVAL;
    *p = c->params;
    return SWE_OK;
}

swe_status swe_set_cell_groups(swe_ctx *c, int64_t n_cells,
                               const uint8_t *group)
{
    if (!c) return SWE_EINVAL;
    if (n_cells < 0 || (n_cells > 0 && !group))
        return fail(c, SWE_EINVAL, "null or negative cell groups");
    c->groups.assign(group, group + n_cells);
    c->wet_band = -1;
    return SWE_OK;
}

swe_status swe_set_wet_cells(swe_ctx *c, int64_t n_cells, const uint8_t *wet,
                             int32_t band)
{
    if (!c) return SWE_EINVAL;
    if (n_cells < 0 || (n_cells > 0 && !wet))
        return fail(c, SWE_EINVAL, "null or negative wet mask");
    if (band < 0 || band > 64)
        return fail(c, SWE_EINVAL, "band must be in [0, 64]");
    c->groups.resize(size_t(n_cells));
    for (int64_t k = 0; k < n_cells; ++k) c->groups[k] = wet[k] ? 1 : 0;
    c->wet_band = n_cells > 0 ? band : -1;
    return SWE_OK;
}

}  // extern "C"

namespace {

// Common part of swe_set_mesh and swe_set_mesh_edges: builds the block mesh
// (edges discovered from the triangles with boundary segments, or taken
// from the caller's edge list) and resets the context to it.
swe_status set_mesh_common(swe_ctx *c, int64_t n_nodes, const double *xy,
                           int64_t n_cells, const int32_t *tri, int64_t n_bnd,
                           const int32_t *bnd_nodes, const int32_t *bnd_tag,
                           const swe::EdgeInput *edges)
{
    if (!c->groups.empty() && int64_t(c->groups.size()) != n_cells) {
        c->groups.clear();
        return fail(c, SWE_EINVAL,
                    "cell groups were set for a different number of cells");
    }
    BlockMesh m;
    std::string err;
    const bool ok = swe::build_block_mesh(
        n_nodes, xy, n_cells, tri, n_bnd, bnd_nodes, bnd_tag,
        c->params.block_cells, c->params.reorder != 0,
        c->groups.empty() ? nullptr : c->groups.data(), c->wet_band,
        SWE_MAX_TAG, m, err, edges);
    c->groups.clear();
    c->wet_band = -1;
    if (!ok) return fail(c, SWE_EMESH, err);
    if (c->ws_owned && c->ws) {
        (void)hipSetDevice(c->device);
        (void)hipFree(c->ws);
    }
    c->ws = nullptr;
    c->ws_bytes = 0;
    c->ws_owned = false;
    c->dev_ready = false;
    c->mesh = std::move(m);
    const size_t nc = size_t(c->mesh.n_cells);
    c->z.assign(nc, 0.0);
    c->man.assign(nc, 0.0);
    c->h.assign(nc, 0.0);
    c->hu.assign(nc, 0.0);
    c->hv.assign(nc, 0.0);
    c->z_dirty = c->man_dirty = c->state_dirty = true;
    c->gm2_dirty = c->bc_dirty = c->clock_dirty = true;
    c->dt_valid = false;
    c->t_host = 0.0;
    c->t_known = true;
    c->step_host = 0;
    c->last_dt_host = 0.0;
    c->step_index = 0;
    c->has_mesh = true;
    return SWE_OK;
}

}  // namespace

extern "C" {

swe_status swe_set_mesh(swe_ctx *c, int64_t n_nodes, const double *xy,
                        int64_t n_cells, const int32_t *tri, int64_t n_bnd,
                        const int32_t *bnd_nodes, const int32_t *bnd_tag)
{
    if (!c) return SWE_EINVAL;
    if (!xy || !tri || n_bnd < 0 || (n_bnd > 0 && (!bnd_nodes || !bnd_tag)))
        return fail(c, SWE_EINVAL, "null mesh array");
    return set_mesh_common(c, n_nodes, xy, n_cells, tri, n_bnd, bnd_nodes,
                           bnd_tag, nullptr);
}

swe_status swe_set_mesh_edges(swe_ctx *c, int64_t n_nodes, const double *xy,
                              int64_t n_cells, const int32_t *tri,
                              int64_t n_edges, const int32_t *edge_nodes,
                              const int32_t *edge_cells,
                              const int32_t *edge_tag)
{
    if (!c) return SWE_EINVAL;
    if (!xy || !tri || n_edges < 0 ||
        (n_edges > 0 && (!edge_nodes || !edge_cells)))
        return fail(c, SWE_EINVAL, "null mesh array");
    swe::EdgeInput in;
    in.n = n_edges;
    in.nodes = edge_nodes;
    in.cells = edge_cells;
    in.tag = edge_tag;
    return set_mesh_common(c, n_nodes, xy, n_cells, tri, 0, nullptr, nullptr,
                           &in);
}

swe_status swe_mesh_info(const swe_ctx *c, swe_mesh_stats *o)
{
    if (!c || !o) return SWE_EINVAL;
    if (!c->has_mesh) return SWE_ENOTREADY;
    const BlockMesh &m = c->mesh;
    o->n_nodes = m.n_nodes;
    o->n_cells = m.n_cells;
    o->n_edges = m.n_edges;
    o->n_boundary_edges = m.n_bnd_edges;
    o->n_blocks = m.n_blocks;
    o->n_block_edges = int64_t(m.be_a.size());
    o->block_cells = m.block_cells;
    o->max_block_edges = m.max_block_edges;
    o->min_inradius = m.min_inradius;
    o->total_area = m.total_area;
    return SWE_OK;
}

swe_status swe_mesh_digest(const swe_ctx *c, uint64_t *digest)
{
    if (!c || !digest) return SWE_EINVAL;
    if (!c->has_mesh) return SWE_ENOTREADY;
    // FNV-1a over the bytes of every array the step kernel reads
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](const void *p, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        for (size_t k = 0; k < n; ++k) {
            h ^= b[k];
            h *= 1099511628211ull;
        }
    };
    const BlockMesh &m = c->mesh;
    auto vec = [&mix](const auto &v) {
        mix(v.data(), v.size() * sizeof(v[0]));
    };
    vec(m.internal_of_user);
    vec(m.area);
    vec(m.inradius);
    vec(m.blk_edge);
    vec(m.be_a);
    vec(m.be_b);
    vec(m.be_nx);
    vec(m.be_ny);
    vec(m.be_len);
    vec(m.bnd_tag);
    vec(m.blk_bnd);
    vec(m.tag_length);
    *digest = h;
    return SWE_OK;
}

swe_status swe_get_cell_order(const swe_ctx *c, int32_t *out)
{
    if (!c || !out) return SWE_EINVAL;
    if (!c->has_mesh) return SWE_ENOTREADY;
    std::memcpy(out, c->mesh.internal_of_user.data(),
                sizeof(int32_t) * size_t(c->mesh.n_cells));
    return SWE_OK;
}

swe_status swe_get_geometry(const swe_ctx *c, double *area, double *inr)
{
    if (!c || !area || !inr) return SWE_EINVAL;
    if (!c->has_mesh) return SWE_ENOTREADY;
    const BlockMesh &m = c->mesh;
    for (int64_t u = 0; u < m.n_cells; ++u) {
        const int32_t i = m.internal_of_user[u];
        area[u] = m.area[i];
        inr[u] = m.inradius[i];
    }
    return SWE_OK;
}

swe_status swe_set_bc(swe_ctx *c, int32_t tag, swe_bc_kind kind, double value)
{
    if (!c) return SWE_EINVAL;
    if (tag < 0 || tag >= SWE_MAX_TAG)
        return fail(c, SWE_EINVAL, "tag out of range");
    if (int(kind) < 0 || int(kind) > 4)
        return fail(c, SWE_EINVAL, "unknown boundary kind");
    if (!std::isfinite(value))
        return fail(c, SWE_EINVAL, "boundary value must be finite");
    if (kind == SWE_BC_FIXED_DEPTH && value < 0.0)
        return fail(c, SWE_EINVAL, "fixed depth must be >= 0");
    c->bc[tag].kind = int32_t(kind);
    c->bc[tag].value = value;
    c->bc_dirty = true;
    return SWE_OK;
}

swe_status swe_set_bathymetry(swe_ctx *c, const double *z, swe_mem mem)
{
    if (!c) return SWE_EINVAL;
    return set_field(c, z, mem, Field::z);
}

swe_status swe_set_manning(swe_ctx *c, const double *n, swe_mem mem)
{
    if (!c) return SWE_EINVAL;
    return set_field(c, n, mem, Field::manning);
}

swe_status swe_set_state(swe_ctx *c, const double *h, const double *hu,
                         const double *hv, swe_mem mem)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    if (!h || !hu || !hv) return fail(c, SWE_EINVAL, "null state array");
    const int64_t nc = c->mesh.n_cells;
    if (mem == SWE_MEM_HOST) {
        for (int64_t u = 0; u < nc; ++u)
            if (!(h[u] >= 0.0) || !std::isfinite(h[u]) ||
                !std::isfinite(hu[u]) || !std::isfinite(hv[u]))
                return fail(c, SWE_ESTATE,
                            "state invalid at cell " + std::to_string(u) +
                                " (need finite values and h >= 0)");
        for (int64_t i = 0; i < nc; ++i) {
            const int32_t u = c->mesh.user_of_internal[i];
            c->h[i] = h[u];
            c->hu[i] = hu[u];
            c->hv[i] = hv[u];
        }
        c->state_dirty = true;
        c->dt_valid = false;
        return SWE_OK;
    }
    if (mem != SWE_MEM_DEVICE) return fail(c, SWE_EINVAL, "bad memory kind");
    if ((st = prepare(c))) return st;
    HIPCHK(c, swe::launch_fill_u32(c->d.flag, 0u, 1, c->stream));
    HIPCHK(c, swe::launch_check_state(h, hu, hv, nc, c->d.flag, c->stream));
    bool bad = false;
    if ((st = check_flag(c, &bad))) return st;
    if (bad)
        return fail(c, SWE_ESTATE, "state invalid (need finite values and "
                                   "h >= 0)");
    const int b = c->cur_buf;
    HIPCHK(c, swe::launch_gather3(h, hu, hv, c->d.h[b], c->d.hu[b],
                                  c->d.hv[b], c->d.user_of_internal, nc,
                                  c->stream));
    c->dt_valid = false;
    c->quiet_dirty = true;
    c->mon_dirty = true;
    return prepare(c);
}

swe_status swe_get_state(swe_ctx *c, double *h, double *hu, double *hv,
                         swe_mem mem)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    if (!h || !hu || !hv) return fail(c, SWE_EINVAL, "null state array");
    if ((st = prepare(c))) return st;
    const int64_t nc = c->mesh.n_cells;
    const int b = c->cur_buf;
    if (mem == SWE_MEM_DEVICE) {
        HIPCHK(c, swe::launch_gather3(c->d.h[b], c->d.hu[b], c->d.hv[b], h,
                                      hu, hv, c->d.internal_of_user, nc,
                                      c->stream));
        return check_health(c);
    }
    if (mem != SWE_MEM_HOST) return fail(c, SWE_EINVAL, "bad memory kind");
    std::vector<double> a(nc), bb(nc), cc(nc);
    HIPCHK(c, hipMemcpyAsync(a.data(), c->d.h[b], nc * 8,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(bb.data(), c->d.hu[b], nc * 8,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(cc.data(), c->d.hv[b], nc * 8,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t u = 0; u < nc; ++u) {
        const int32_t i = c->mesh.internal_of_user[u];
        h[u] = a[i];
        hu[u] = bb[i];
        hv[u] = cc[i];
    }
    return check_health(c);
}

swe_status swe_set_time(swe_ctx *c, double t, int64_t step)
{
    if (!c) return SWE_EINVAL;
    if (!std::isfinite(t)) return fail(c, SWE_EINVAL, "time must be finite");
    c->t_host = t;
    c->t_known = true;
    c->step_host = step;
    c->clock_dirty = true;
    return SWE_OK;
}

swe_status swe_get_time(swe_ctx *c, double *t, double *last_dt,
                        int64_t *step)
{
    if (!c) return SWE_EINVAL;
    if (c->dev_ready && !c->t_known) {
        Clock ck;
        swe_status st = read_clock(c, &ck);
        if (st) return st;
    }
    if (t) *t = c->t_host;
    if (last_dt) *last_dt = c->last_dt_host;
    if (step) *step = c->step_host;
    return SWE_OK;
}

}  // extern "C"

namespace swe {

// Threads per block of the step: block_threads, or with 0 one per cell,
// two per cell on a mesh of fewer blocks than the GPU has compute units,
// whose step is bound by each block's chain of dependent loads and
// arithmetic rather than by throughput (the 4 000-cell canal: 9.5 -> 8.7 us
// per step); the results are the same bits either way.
int step_threads(const swe_ctx *c)
{
    if (c->params.block_threads != 0) return c->params.block_threads;
    const int B = c->mesh.block_cells;
    return c->mesh.n_blocks < 256 && B <= 512 ? 2 * B : B;
}

swe_status ctx_prepare(swe_ctx *c) { return prepare(c); }

swe_status ctx_fail(swe_ctx *c, swe_status st, const std::string &msg)
{
    return fail(c, st, msg);
}

swe_status ctx_read_clock(swe_ctx *c) 
{
    Clock ck;
    return read_clock(c, &ck);
}

StepArgs ctx_step_args(swe_ctx *c, double t_end)
{
    const BlockMesh &m = c->mesh;
    StepArgs a{};
    a.blk_edge = c->d.blk_edge;
    a.be_a = c->d.be_a;
    a.be_b = c->d.be_b;
    a.be_nx = c->d.be_nx;
    a.be_ny = c->d.be_ny;
    a.be_len = c->d.be_len;
    a.z = c->d.z;
    a.gm2 = c->d.gm2;
    a.area = c->d.area;
    a.inradius = c->d.inr;
    a.bc = c->d.bc;
    a.clock = c->d.clock;
    a.ledger = c->d.ledger;
    a.quiet = c->d.quiet;
    a.run = c->d.run;
    a.act = c->d.act;
    a.store_all = c->params.store_all;
    if (c->params.monitors) a.mon = c->d.mon;
    a.g = c->params.g;
    a.cfl = c->params.cfl;
    a.h_dry = c->params.h_dry;
    a.dt_max = c->params.dt_max;
    a.t_end = t_end;
    a.n_cells = int32_t(m.n_cells);
    a.n_blocks = m.n_blocks;
    a.blk_base = 0;
    return a;
}

swe_status ctx_step_between(swe_ctx *c, const double *const in[3],
                            double *const out[3], double dt,
                            uint8_t *run_log, double *r_out)
{
    StepArgs a = ctx_step_args(c, INFINITY);
    a.h0 = in[0];
    a.hu0 = in[1];
    a.hv0 = in[2];
    a.h1 = out[0];
    a.hu1 = out[1];
    a.hv1 = out[2];
    a.cfl = INFINITY;   // dt = min(cfl * min R/s, dt_max) = dt exactly
    a.dt_max = dt;
    a.fresh_out = 1;    // `out` need not hold the state before `in`
    a.run_log = run_log;
    a.r_out = r_out;
    a.mon = nullptr;
    a.cur = c->cur_slot;
    a.step_index = c->step_index;
    const int threads = step_threads(c);
    hipError_t e = launch_step(a, c->mesh.block_cells, threads,
                               c->params.load_schedule, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "step kernel launch");
    c->cur_slot = (c->cur_slot + 1) % 3;
    ++c->step_index;
    c->t_known = false;
    return SWE_OK;
}

swe_status ctx_dt_buffer(swe_ctx *c, int64_t n)
{
    if (n <= c->dt_cap) return SWE_OK;
    if (c->dt_dev) HIPCHK(c, hipFree(c->dt_dev));
    c->dt_dev = nullptr;
    c->dt_cap = 0;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, size_t(n) * 8);
    if (e != hipSuccess)
        return fail(c, SWE_ENOMEM, "time-step buffer: " +
                                       std::string(hipGetErrorString(e)));
    c->dt_dev = (double *)p;
    c->dt_cap = n;
    return SWE_OK;
}

swe_status ctx_enqueue(swe_ctx *c, StepArgs &a, int64_t n,
                       const double *dt_fixed, double *dt_log,
                       double *slots, size_t stride, uint8_t *run_log,
                       double *r_log)
{
    const BlockMesh &m = c->mesh;
    const size_t nc = size_t(m.n_cells);
    const int threads = step_threads(c);
    if (!dt_fixed && !dt_log && !slots && !run_log && !r_log) {
        // plain steps: one launch each, or graph replays (graph_steps)
        const StepBuffers b{{c->d.h[0], c->d.h[1]},
                            {c->d.hu[0], c->d.hu[1]},
                            {c->d.hv[0], c->d.hv[1]}};
        hipError_t e = enqueue_steps(
            a, b, c->cur_buf, c->cur_slot, c->step_index, n,
            StepLaunch{m.block_cells, threads, c->params.load_schedule},
            &c->graph, c->params.graph_steps, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "step launch");
        c->t_known = false;
        return SWE_OK;
    }
    int64_t logged = 0;   // dt_log entries written
    for (int64_t k = 0; k < n; ++k) {
        if (slots) {
            double *u = slots + size_t(k) * stride;
            double *w = u + stride;
            a.h0 = u;
            a.hu0 = u + nc;
            a.hv0 = u + 2 * nc;
            a.h1 = w;
            a.hu1 = w + nc;
            a.hv1 = w + 2 * nc;
            a.fresh_out = 1;   // a fresh slot holds no earlier state
        } else {
            const int b = c->cur_buf;
            a.h0 = c->d.h[b];
            a.hu0 = c->d.hu[b];
            a.hv0 = c->d.hv[b];
            a.h1 = c->d.h[b ^ 1];
            a.hu1 = c->d.hu[b ^ 1];
            a.hv1 = c->d.hv[b ^ 1];
        }
        a.cur = c->cur_slot;
        a.step_index = c->step_index;
        a.run_log = run_log ? run_log + size_t(k) * size_t(m.n_blocks)
                            : nullptr;
        a.r_out = r_log ? r_log + size_t(k) * 3 * nc : nullptr;
        if (dt_fixed) {
            // dt = min(cfl * min R/s, dt_max) = dt_fixed[k] exactly
            a.cfl = INFINITY;
            a.dt_max = dt_fixed[k];
            a.t_end = INFINITY;
        }
        hipError_t e = launch_step(a, m.block_cells, threads,
                                   c->params.load_schedule, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "step kernel launch");
        // the clock keeps the time steps of the last 8 step indices: copy
        // them out whenever the ring is about to wrap, and at the end
        const long long q = c->step_index;
        if (dt_log && (((q + 1) & 7) == 0 || k + 1 == n)) {
            int64_t j = logged;
            while (j <= k) {
                const int slot = int((q - k + j) & 7);
                const int64_t run = std::min<int64_t>(k - j + 1, 8 - slot);
                HIPCHK(c, hipMemcpyAsync(dt_log + j,
                                         &c->d.clock->dt_ring[slot],
                                         size_t(run) * 8,
                                         hipMemcpyDeviceToDevice, c->stream));
                j += run;
            }
            logged = k + 1;
        }
        if (!slots) c->cur_buf ^= 1;
        c->cur_slot = (c->cur_slot + 1) % 3;
        ++c->step_index;
    }
    c->t_known = false;
    return SWE_OK;
}

swe_status ctx_advance_dt_check(swe_ctx *c, int64_t n, const double *dt)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    if (n < 0) return fail(c, SWE_EINVAL, "negative step count");
    if (dt)
        for (int64_t k = 0; k < n; ++k)
            if (!(dt[k] >= 0.0) || !std::isfinite(dt[k]))
                return fail(c, SWE_EINVAL,
                            "time step " + std::to_string(k) +
                                " must be finite and >= 0");
    return SWE_OK;
}

swe_status ctx_advance_dt(swe_ctx *c, int64_t n, const double *dt,
                          double *dt_out, double *log)
{
    swe_status st;
    if (!c->t_known) {
        Clock ck;
        if ((st = read_clock(c, &ck))) return st;
    }
    StepArgs a = ctx_step_args(c, INFINITY);
    if ((st = ctx_enqueue(c, a, n, dt, dt_out ? log : nullptr))) return st;
    if (dt_out)
        HIPCHK(c, hipMemcpyAsync(dt_out, log, size_t(n) * 8,
                                 hipMemcpyDeviceToHost, c->stream));
    Clock ck;
    return read_clock(c, &ck);
}

}  // namespace swe

extern "C" {

swe_status swe_advance(swe_ctx *c, int64_t max_steps, double t_end,
                       int64_t *steps_done, double *t_now)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    if (max_steps < 0) return fail(c, SWE_EINVAL, "max_steps < 0");
    if (std::isnan(t_end)) return fail(c, SWE_EINVAL, "t_end is NaN");
    if ((st = prepare(c))) return st;
    Clock ck;
    if (!c->t_known) {
        if ((st = read_clock(c, &ck))) return st;
    }
    const int64_t steps0 = c->step_host;
    swe::StepArgs a = swe::ctx_step_args(c, t_end);
    if (std::isinf(t_end) && t_end > 0) {
        if ((st = swe::ctx_enqueue(c, a, max_steps, nullptr, nullptr)))
            return st;
        c->step_host = steps0 + max_steps;
        if (t_now) {
            if ((st = read_clock(c, &ck))) return st;
            *t_now = c->t_host;
        }
        if (steps_done) *steps_done = max_steps;
        return SWE_OK;
    }
    int64_t launched = 0;
    while (launched < max_steps && c->t_host < t_end) {
        const int64_t n = std::min<int64_t>(c->params.check_every,
                                            max_steps - launched);
        if ((st = swe::ctx_enqueue(c, a, n, nullptr, nullptr))) return st;
        launched += n;
        if ((st = read_clock(c, &ck))) return st;
    }
    if (steps_done) *steps_done = c->step_host - steps0;
    if (t_now) *t_now = c->t_host;
    return SWE_OK;
}

swe_status swe_advance_dt(swe_ctx *c, int64_t n, const double *dt,
                          double *dt_out)
{
    swe_status st = swe::ctx_advance_dt_check(c, n, dt);
    if (st != SWE_OK || n == 0) return st;
    if ((st = prepare(c))) return st;
    double *log = nullptr;
    if (dt_out) {
        if ((st = swe::ctx_dt_buffer(c, n))) return st;
        log = c->dt_dev;
    }
    return swe::ctx_advance_dt(c, n, dt, dt_out, log);
}

swe_status swe_get_diagnostics(swe_ctx *c, double *mass, double *ledger,
                               int64_t *n_wet)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    if ((st = prepare(c))) return st;
    const int64_t nc = c->mesh.n_cells;
    const int b = c->cur_buf;
    HIPCHK(c, swe::launch_diag(c->d.h[b], c->d.area, nc, c->params.h_dry,
                               c->d.part_mass, c->d.part_wet, kDiagParts,
                               c->stream));
    std::vector<double> pm(kDiagParts);
    std::vector<unsigned long long> pw(kDiagParts);
    std::vector<double> led(c->mesh.n_blocks);
    HIPCHK(c, hipMemcpyAsync(pm.data(), c->d.part_mass, kDiagParts * 8,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(pw.data(), c->d.part_wet, kDiagParts * 8,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(led.data(), c->d.ledger, led.size() * 8,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double s = 0.0, l = 0.0;
    unsigned long long w = 0;
    for (int k = 0; k < kDiagParts; ++k) {
        s += pm[k];
        w += pw[k];
    }
    for (double x : led) l += x;
    if (mass) *mass = s;
    if (ledger) *ledger = l;
    if (n_wet) *n_wet = int64_t(w);
    return check_health(c);
}

swe_status swe_get_activity(swe_ctx *c, int64_t *blocks, int64_t *cells)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    if ((st = prepare(c))) return st;
    const BlockMesh &m = c->mesh;
    const int64_t nb = m.n_blocks, B = m.block_cells;
    // the kernel's test: dormant skipping on, the mark of this step's
    // parity clear, and not the block that advances the clock
    const bool all = c->params.store_all != 0;
    std::vector<uint32_t> mark(size_t(nb), 1u);
    if (!all) {
        HIPCHK(c, hipMemcpyAsync(mark.data(),
                                 c->d.run + size_t(c->step_index & 1) * nb,
                                 size_t(nb) * 4, hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    int64_t b = 0, n = 0;
    for (int64_t k = 0; k < nb; ++k)
        if (mark[size_t(k)] || k == 0) {
            ++b;
            n += std::min<int64_t>(B, m.n_cells - k * B);
        }
    if (blocks) *blocks = b;
    if (cells) *cells = n;
    return check_health(c);
}

swe_status swe_reset_monitors(swe_ctx *c)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    c->mon_dirty = true;
    if (!c->params.monitors) return SWE_OK;
    return prepare(c);
}

swe_status swe_get_discharge(swe_ctx *c, int32_t tag, double *rate,
                             double *volume)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    if (tag < 0 || tag >= SWE_MAX_TAG)
        return fail(c, SWE_EINVAL, "tag out of range");
    if (!c->params.monitors)
        return fail(c, SWE_ENOTREADY, "monitors are off (swe_params.monitors)");
    if ((st = prepare(c))) return st;
    const std::vector<int32_t> &bt = c->mesh.bnd_tag;
    std::vector<double> r(bt.size()), v(bt.size());
    if (!bt.empty()) {
        HIPCHK(c, hipMemcpyAsync(r.data(), c->d.mon_rate, bt.size() * 8,
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(v.data(), c->d.mon_vol, bt.size() * 8,
                                 hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double sr = 0.0, sv = 0.0;
    for (size_t k = 0; k < bt.size(); ++k)
        if (bt[k] == tag) {
            sr += r[k];
            sv += v[k];
        }
    if (rate) *rate = sr;
    if (volume) *volume = sv;
    return SWE_OK;
}

swe_status swe_discharge_async(swe_ctx *c, double *out)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    if (!out) return fail(c, SWE_EINVAL, "null output array");
    if (!c->params.monitors)
        return fail(c, SWE_ENOTREADY, "monitors are off (swe_params.monitors)");
    if (c->copy_pending)
        return fail(c, SWE_ENOTREADY,
                    "an asynchronous discharge copy is pending "
                    "(swe_discharge_wait)");
    if ((st = prepare(c))) return st;
    if (!c->side) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_step,
                                          hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_copy,
                                          hipEventDisableTiming));
    }
    // the side stream follows every step enqueued so far; the next steps
    // wait for its per-tag sums (a few microseconds), not for the copy
    HIPCHK(c, hipEventRecord(c->ev_step, c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->side, c->ev_step, 0));
    HIPCHK(c, swe::launch_discharge_tags(c->d.mon_rate, c->d.mon_vol,
                                         c->d.tag_ptr, c->d.tag_slot,
                                         SWE_MAX_TAG, c->d.tag_out, c->side));
    HIPCHK(c, hipEventRecord(c->ev_step, c->side));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_step, 0));
    HIPCHK(c, hipMemcpyAsync(out, c->d.tag_out, 2 * SWE_MAX_TAG * 8,
                             hipMemcpyDeviceToHost, c->side));
    HIPCHK(c, hipEventRecord(c->ev_copy, c->side));
    c->copy_pending = true;
    return SWE_OK;
}

swe_status swe_discharge_wait(swe_ctx *c, int32_t block, int32_t *done)
{
    if (!c) return SWE_EINVAL;
    if (done) *done = 1;
    if (!c->copy_pending) return SWE_OK;
    if (block) {
        HIPCHK(c, hipEventSynchronize(c->ev_copy));
    } else {
        const hipError_t e = hipEventQuery(c->ev_copy);
        if (e == hipErrorNotReady) {
            if (done) *done = 0;
            return SWE_OK;
        }
        HIPCHK(c, e);
    }
    c->copy_pending = false;
    return SWE_OK;
}

swe_status swe_get_envelope(swe_ctx *c, double *h_max, double *t_wet,
                            swe_mem mem)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    if (!h_max || !t_wet) return fail(c, SWE_EINVAL, "null envelope array");
    if (!c->params.monitors)
        return fail(c, SWE_ENOTREADY, "monitors are off (swe_params.monitors)");
    if ((st = prepare(c))) return st;
    const int64_t nc = c->mesh.n_cells;
    if (mem == SWE_MEM_DEVICE) {
        HIPCHK(c, swe::launch_gather1(c->d.h_max, h_max,
                                      c->d.internal_of_user, nc, c->stream));
        HIPCHK(c, swe::launch_gather1(c->d.t_wet, t_wet,
                                      c->d.internal_of_user, nc, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return SWE_OK;
    }
    if (mem != SWE_MEM_HOST) return fail(c, SWE_EINVAL, "bad memory kind");
    std::vector<double> a(nc), b(nc);
    HIPCHK(c, hipMemcpyAsync(a.data(), c->d.h_max, nc * 8,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(b.data(), c->d.t_wet, nc * 8,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t u = 0; u < nc; ++u) {
        const int32_t i = c->mesh.internal_of_user[u];
        h_max[u] = a[i];
        t_wet[u] = b[i];
    }
    return SWE_OK;
}

swe_status swe_workspace_bytes(const swe_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return SWE_EINVAL;
    if (!c->has_mesh) return SWE_ENOTREADY;
    *bytes = layout(c->mesh, nullptr, nullptr);
    return SWE_OK;
}

swe_status swe_bind_workspace(swe_ctx *c, void *ptr, size_t bytes)
{
    swe_status st = require_mesh(c);
    if (st != SWE_OK) return st;
    if (c->dev_ready)
        return fail(c, SWE_ENOTREADY,
                    "workspace must be bound before the first device use");
    if (!ptr || (uintptr_t(ptr) & 255u))
        return fail(c, SWE_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = layout(c->mesh, nullptr, nullptr);
    if (bytes < need)
        return fail(c, SWE_ENOMEM, "workspace of " + std::to_string(bytes) +
                                       " bytes, need " + std::to_string(need));
    c->ws = ptr;
    c->ws_bytes = bytes;
    c->ws_owned = false;
    return SWE_OK;
}

}  // extern "C"
