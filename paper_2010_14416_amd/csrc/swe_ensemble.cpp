// Batched ensemble (swe_ens_* of include/swe.h): the meshes of many
// configured contexts, laid end to end in one device workspace and advanced
// by one launch of the step kernel per step, each member with its own time
// step and clock. The many sampled runs behind the flood lines of
// sec. 6.4.3 are small meshes each; batched, they fill the GPU that a single
// one leaves mostly idle.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "swe.h"
#include "swe_ctx.hpp"
#include "swe_device.hpp"
#include "swe_mesh.hpp"

using swe::BcEntry;
using swe::Clock;

struct swe_ens {
    int device = 0;
    hipStream_t stream = nullptr;
    swe_params params{};
    std::string err;
    int32_t n_members = 0;
    int32_t block_cells = 256;
    // per member: first internal cell (a multiple of block_cells), cells,
    // first block, internal index of each user cell, start time and steps
    std::vector<int64_t> cell_off, n_cells, blk_off;
    std::vector<std::vector<int32_t>> internal_of_user;
    std::vector<double> t_start;
    std::vector<int64_t> steps_start;
    // concatenated inputs, uploaded at the first device use
    int64_t total_cells = 0, total_blocks = 0;
    std::vector<int32_t> blk_edge, be_a, be_b, blk_member, member_end;
    std::vector<double> be_nx, be_ny, be_len, area, inr, z, man, h, hu, hv;
    std::vector<BcEntry> bc_slot;
    // device
    bool dev_ready = false;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    struct {
        double *h[2], *hu[2], *hv[2];
        double *z, *man, *gm2, *area, *inr;
        int32_t *blk_edge, *be_a, *be_b, *blk_member, *member_end;
        double *be_nx, *be_ny, *be_len;
        BcEntry *bc;
        Clock *clock;
        double *ledger;
        int32_t *quiet;
        uint32_t *run;
        unsigned long long *act;
        double *t_end;
    } d{};
    std::vector<double> t_end_host;   // as last uploaded
    int cur_buf = 0;
    int cur_slot = 0;
    long long step_index = 0;
    swe::StepGraph graph;   // captured step runs (graph_steps > 0)
};

namespace {

thread_local std::string g_ens_create_error;

swe_status efail(swe_ens *e, swe_status s, const std::string &msg)
{
    if (e) e->err = msg;
    return s;
}

#define ENSCHK(ens, call)                                                  \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess)                                              \
            return efail(ens, SWE_EDEVICE,                                 \
                         std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t ens_layout(swe_ens *e, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const size_t nc = size_t(e->total_cells), nb = size_t(e->total_blocks);
    const size_t nbe = e->be_a.size();
    const size_t nbnd = std::max<size_t>(e->bc_slot.size(), 1);
    const size_t nm = size_t(e->n_members);
    for (int k = 0; k < 2; ++k) {
        e->d.h[k] = (double *)take(nc * 8);
        e->d.hu[k] = (double *)take(nc * 8);
        e->d.hv[k] = (double *)take(nc * 8);
    }
    e->d.z = (double *)take(nc * 8);
    e->d.man = (double *)take(nc * 8);
    e->d.gm2 = (double *)take(nc * 8);
    e->d.area = (double *)take(nc * 8);
    e->d.inr = (double *)take(nc * 8);
    e->d.blk_edge = (int32_t *)take((nb + 1) * 4);
    e->d.be_a = (int32_t *)take(nbe * 4);
    e->d.be_b = (int32_t *)take(nbe * 4);
    e->d.blk_member = (int32_t *)take(nb * 4);
    e->d.member_end = (int32_t *)take(nm * 4);
    e->d.be_nx = (double *)take(nbe * 8);
    e->d.be_ny = (double *)take(nbe * 8);
    e->d.be_len = (double *)take(nbe * 8);
    e->d.bc = (BcEntry *)take(nbnd * sizeof(BcEntry));
    e->d.clock = (Clock *)take(nm * sizeof(Clock));
    e->d.ledger = (double *)take(nb * 8);
    e->d.quiet = (int32_t *)take(nb * 4);
    e->d.act = (unsigned long long *)take(nb * (e->block_cells / 64) * 8);
    e->d.run = (uint32_t *)take(2 * nb * 4);
    e->d.t_end = (double *)take(nm * 8);
    return off;
}

// The member's current field `host` (internal order) unless the device
// holds a newer copy at `dev`.
swe_status member_field(swe_ens *e, swe_ctx *c, const std::vector<double> &host,
                        bool host_newer, const double *dev, double *out)
{
    const size_t n = size_t(c->mesh.n_cells);
    if (c->dev_ready && !host_newer) {
        ENSCHK(e, hipSetDevice(c->device));
        ENSCHK(e, hipMemcpyAsync(out, dev, n * 8, hipMemcpyDeviceToHost,
                                 c->stream));
        ENSCHK(e, hipStreamSynchronize(c->stream));
    } else {
        std::copy(host.begin(), host.end(), out);
    }
    return SWE_OK;
}

template <typename T>
swe_status up(swe_ens *e, T *dst, const T *src, size_t n)
{
    if (n == 0) return SWE_OK;
    ENSCHK(e, hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice,
                             e->stream));
    return SWE_OK;
}

swe_status ens_prepare(swe_ens *e)
{
    if (e->dev_ready) return SWE_OK;
    ENSCHK(e, hipSetDevice(e->device));
    const size_t need = ens_layout(e, nullptr);
    if (!e->ws) {
        void *p = nullptr;
        hipError_t er = hipMalloc(&p, need);
        if (er != hipSuccess)
            return efail(e, SWE_ENOMEM,
                         "device allocation of " + std::to_string(need) +
                             " bytes failed: " + hipGetErrorString(er));
        e->ws = p;
        e->ws_bytes = need;
        e->ws_owned = true;
    }
    ens_layout(e, (char *)e->ws);
    const size_t nc = size_t(e->total_cells), nb = size_t(e->total_blocks);
    const size_t nbe = e->be_a.size();
    swe_status st;
    if ((st = up(e, e->d.h[0], e->h.data(), nc))) return st;
    if ((st = up(e, e->d.hu[0], e->hu.data(), nc))) return st;
    if ((st = up(e, e->d.hv[0], e->hv.data(), nc))) return st;
    if ((st = up(e, e->d.z, e->z.data(), nc))) return st;
    if ((st = up(e, e->d.man, e->man.data(), nc))) return st;
    if ((st = up(e, e->d.area, e->area.data(), nc))) return st;
    if ((st = up(e, e->d.inr, e->inr.data(), nc))) return st;
    if ((st = up(e, e->d.blk_edge, e->blk_edge.data(), nb + 1))) return st;
    if ((st = up(e, e->d.be_a, e->be_a.data(), nbe))) return st;
    if ((st = up(e, e->d.be_b, e->be_b.data(), nbe))) return st;
    if ((st = up(e, e->d.be_nx, e->be_nx.data(), nbe))) return st;
    if ((st = up(e, e->d.be_ny, e->be_ny.data(), nbe))) return st;
    if ((st = up(e, e->d.be_len, e->be_len.data(), nbe))) return st;
    if ((st = up(e, e->d.blk_member, e->blk_member.data(), nb))) return st;
    if ((st = up(e, e->d.member_end, e->member_end.data(),
                 size_t(e->n_members))))
        return st;
    if ((st = up(e, e->d.bc, e->bc_slot.data(), e->bc_slot.size())))
        return st;
    e->t_end_host.assign(size_t(e->n_members), INFINITY);
    if ((st = up(e, e->d.t_end, e->t_end_host.data(), size_t(e->n_members))))
        return st;
    ENSCHK(e, swe::launch_gm2(e->d.man, e->d.gm2, int64_t(nc), e->params.g,
                              e->stream));
    ENSCHK(e, swe::launch_fill_f64(e->d.ledger, 0.0, int64_t(nb), e->stream));
    ENSCHK(e, swe::launch_fill_u32((unsigned *)e->d.quiet, 0u, int64_t(nb),
                                   e->stream));
    ENSCHK(e, swe::launch_fill_u32(e->d.run, 1u, 2 * int64_t(nb), e->stream));
    ENSCHK(e, swe::launch_fill_u32((unsigned *)e->d.act, 0u,
                                   int64_t(nb) * e->block_cells / 32,
                                   e->stream));
    for (int32_t m = 0; m < e->n_members; ++m) {
        Clock *ck = e->d.clock + m;
        const int64_t c0 = e->cell_off[m];
        ENSCHK(e, swe::launch_clock_set(ck, e->t_start[m], e->steps_start[m],
                                        e->step_index, e->stream));
        ENSCHK(e, swe::launch_min_rs(e->d.h[0] + c0, e->d.hu[0] + c0,
                                     e->d.hv[0] + c0, e->d.inr + c0,
                                     e->n_cells[m], e->params.g,
                                     e->params.h_dry, ck, 0, e->stream));
    }
    ENSCHK(e, hipStreamSynchronize(e->stream));
    e->cur_buf = 0;
    e->cur_slot = 0;
    e->dev_ready = true;
    return SWE_OK;
}

swe_status read_member_clock(swe_ens *e, int32_t m, Clock *out)
{
    ENSCHK(e, hipSetDevice(e->device));
    ENSCHK(e, hipMemcpyAsync(out, e->d.clock + m, sizeof(Clock),
                             hipMemcpyDeviceToHost, e->stream));
    ENSCHK(e, hipStreamSynchronize(e->stream));
    if (out->health) {
        std::string why = (out->health & 1u) ? "non-finite state"
                                             : "unbounded time step";
        return efail(e, SWE_ENUMERIC,
                     "member " + std::to_string(m) + ": " + why +
                         " at step " + std::to_string(out->bad_step));
    }
    return SWE_OK;
}

}  // namespace

extern "C" {

swe_status swe_ens_create(swe_ens **out, swe_ctx *const *members,
                          int32_t n_members)
{
    if (!out) return SWE_EINVAL;
    *out = nullptr;
    if (!members || n_members < 1) {
        g_ens_create_error = "need at least one member";
        return SWE_EINVAL;
    }
    for (int32_t m = 0; m < n_members; ++m)
        if (!members[m] || !members[m]->has_mesh) {
            g_ens_create_error =
                "member " + std::to_string(m) + " has no mesh";
            return SWE_ENOTREADY;
        }
    const swe_params &p0 = members[0]->params;
    for (int32_t m = 1; m < n_members; ++m) {
        const swe_params &p = members[m]->params;
        if (p.g != p0.g || p.cfl != p0.cfl || p.h_dry != p0.h_dry ||
            p.dt_max != p0.dt_max ||
            members[m]->mesh.block_cells != members[0]->mesh.block_cells ||
            members[m]->device != members[0]->device) {
            g_ens_create_error =
                "member " + std::to_string(m) +
                " differs from member 0 in g, cfl, h_dry, dt_max, block "
                "size or device";
            return SWE_EINVAL;
        }
    }
    swe_ens *e = new (std::nothrow) swe_ens();
    if (!e) {
        g_ens_create_error = "out of memory";
        return SWE_ENOMEM;
    }
    e->device = members[0]->device;
    e->params = p0;
    e->n_members = n_members;
    const int32_t B = members[0]->mesh.block_cells;
    e->block_cells = B;
    // offsets
    int64_t cells = 0, blocks = 0, recs = 0, slots = 0;
    for (int32_t m = 0; m < n_members; ++m) {
        const swe::BlockMesh &M = members[m]->mesh;
        e->cell_off.push_back(cells);
        e->n_cells.push_back(M.n_cells);
        e->blk_off.push_back(blocks);
        cells += int64_t(M.n_blocks) * B;
        blocks += M.n_blocks;
        recs += int64_t(M.be_a.size());
        slots += int64_t(M.bnd_tag.size());
    }
    // the step addresses its arrays with 32-bit byte offsets
    if (cells >= (int64_t(1) << 29) || slots >= (int64_t(1) << 30) ||
        recs >= (int64_t(1) << 30)) {
        delete e;
        g_ens_create_error = "ensemble too large: fewer than 2^29 cells "
                             "and 2^30 block-edge records in total";
        return SWE_EINVAL;
    }
    e->total_cells = cells;
    e->total_blocks = blocks;
    const size_t nc = size_t(cells);
    e->area.assign(nc, 1.0);
    e->inr.assign(nc, 1.0);
    e->z.assign(nc, 0.0);
    e->man.assign(nc, 0.0);
    e->h.assign(nc, 0.0);
    e->hu.assign(nc, 0.0);
    e->hv.assign(nc, 0.0);
    e->blk_edge.reserve(size_t(blocks) + 1);
    e->be_a.reserve(size_t(recs));
    e->be_b.reserve(size_t(recs));
    e->be_nx.reserve(size_t(recs));
    e->be_ny.reserve(size_t(recs));
    e->be_len.reserve(size_t(recs));
    e->bc_slot.reserve(size_t(slots));
    int64_t rec_off = 0, slot_off = 0;
    for (int32_t m = 0; m < n_members; ++m) {
        swe_ctx *c = members[m];
        const swe::BlockMesh &M = c->mesh;
        const int64_t c0 = e->cell_off[m];
        const size_t n = size_t(M.n_cells);
        std::copy(M.area.begin(), M.area.end(), e->area.begin() + c0);
        std::copy(M.inradius.begin(), M.inradius.end(), e->inr.begin() + c0);
        swe_status st;
        if ((st = member_field(e, c, c->z, c->z_dirty, c->d.z,
                               e->z.data() + c0)) ||
            (st = member_field(e, c, c->man, c->man_dirty, c->d.man,
                               e->man.data() + c0)) ||
            (st = member_field(e, c, c->h, c->state_dirty, c->d.h[c->cur_buf],
                               e->h.data() + c0)) ||
            (st = member_field(e, c, c->hu, c->state_dirty,
                               c->d.hu[c->cur_buf], e->hu.data() + c0)) ||
            (st = member_field(e, c, c->hv, c->state_dirty,
                               c->d.hv[c->cur_buf], e->hv.data() + c0))) {
            g_ens_create_error = "member " + std::to_string(m) + ": " + e->err;
            delete e;
            return st;
        }
        // time: the host copy, or the member's device clock
        double t = c->t_host;
        int64_t steps = c->step_host;
        if (c->dev_ready && !c->t_known) {
            double ldt;
            if ((st = swe_get_time(c, &t, &ldt, &steps))) {
                g_ens_create_error =
                    "member " + std::to_string(m) + ": " + c->err;
                delete e;
                return st;
            }
        }
        e->t_start.push_back(t);
        e->steps_start.push_back(steps);
        // blocks and records, with indices moved to the ensemble's ranges
        for (int32_t b = 0; b < M.n_blocks; ++b) {
            e->blk_edge.push_back(int32_t(rec_off + M.blk_edge[b]));
            e->blk_member.push_back(int32_t(uint32_t(m) |
                                            (b == 0 ? 0x80000000u : 0u)));
        }
        auto move = [&](int32_t v) {
            const uint32_t u = uint32_t(v);
            if (u & swe::kSideLocal) return v;
            if (u & swe::kSideBoundary)
                return int32_t(swe::kSideBoundary |
                               uint32_t((u & 0x3fffffffu) + slot_off));
            return int32_t(v + c0);
        };
        for (size_t r = 0; r < M.be_a.size(); ++r) {
            e->be_a.push_back(move(M.be_a[r]));
            e->be_b.push_back(move(M.be_b[r]));
        }
        e->be_nx.insert(e->be_nx.end(), M.be_nx.begin(), M.be_nx.end());
        e->be_ny.insert(e->be_ny.end(), M.be_ny.begin(), M.be_ny.end());
        e->be_len.insert(e->be_len.end(), M.be_len.begin(), M.be_len.end());
        // boundary conditions per slot, with the member's inflow per length
        for (int32_t tag : M.bnd_tag) {
            BcEntry b = c->bc[tag];
            const double L = M.tag_length[tag];
            b.q = (b.kind == SWE_BC_INFLOW && L > 0.0) ? b.value / L : 0.0;
            e->bc_slot.push_back(b);
        }
        e->member_end.push_back(int32_t(c0 + int64_t(n)));
        e->internal_of_user.push_back(M.internal_of_user);
        rec_off += int64_t(M.be_a.size());
        slot_off += int64_t(M.bnd_tag.size());
    }
    e->blk_edge.push_back(int32_t(rec_off));
    *out = e;
    return SWE_OK;
}

void swe_ens_destroy(swe_ens *e)
{
    if (!e) return;
    if (e->ws_owned && e->ws) {
        (void)hipSetDevice(e->device);
        (void)hipFree(e->ws);
    }
    delete e;
}

const char *swe_ens_last_error(const swe_ens *e)
{
    return e ? e->err.c_str() : g_ens_create_error.c_str();
}

swe_status swe_ens_set_stream(swe_ens *e, void *stream)
{
    if (!e) return SWE_EINVAL;
    e->stream = (hipStream_t)stream;
    return SWE_OK;
}

swe_status swe_ens_workspace_bytes(swe_ens *e, size_t *bytes)
{
    if (!e || !bytes) return SWE_EINVAL;
    if (e->dev_ready) {
        *bytes = e->ws_bytes;
        return SWE_OK;
    }
    auto saved = e->d;
    *bytes = ens_layout(e, nullptr);
    e->d = saved;
    return SWE_OK;
}

swe_status swe_ens_bind_workspace(swe_ens *e, void *ptr, size_t bytes)
{
    if (!e) return SWE_EINVAL;
    if (e->dev_ready)
        return efail(e, SWE_ENOTREADY,
                     "workspace must be bound before the first device use");
    if (!ptr || (uintptr_t(ptr) & 255u))
        return efail(e, SWE_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    swe_ens_workspace_bytes(e, &need);
    if (bytes < need)
        return efail(e, SWE_ENOMEM, "workspace of " + std::to_string(bytes) +
                                        " bytes, need " +
                                        std::to_string(need));
    e->ws = ptr;
    e->ws_bytes = bytes;
    e->ws_owned = false;
    return SWE_OK;
}

swe_status swe_ens_advance(swe_ens *e, int64_t steps, const double *t_end)
{
    if (!e) return SWE_EINVAL;
    if (steps < 0) return efail(e, SWE_EINVAL, "negative step count");
    swe_status st = ens_prepare(e);
    if (st) return st;
    ENSCHK(e, hipSetDevice(e->device));
    const size_t nm = size_t(e->n_members);
    bool changed = false;
    for (size_t m = 0; m < nm; ++m) {
        const double te = t_end ? t_end[m] : INFINITY;
        if (std::isnan(te))
            return efail(e, SWE_EINVAL,
                         "t_end of member " + std::to_string(m) + " is NaN");
        if (!(te == e->t_end_host[m])) changed = true;
    }
    if (changed) {
        for (size_t m = 0; m < nm; ++m)
            e->t_end_host[m] = t_end ? t_end[m] : INFINITY;
        ENSCHK(e, hipMemcpyAsync(e->d.t_end, e->t_end_host.data(), nm * 8,
                                 hipMemcpyHostToDevice, e->stream));
        ENSCHK(e, hipStreamSynchronize(e->stream));
    }
    swe::StepArgs a{};
    a.blk_edge = e->d.blk_edge;
    a.be_a = e->d.be_a;
    a.be_b = e->d.be_b;
    a.be_nx = e->d.be_nx;
    a.be_ny = e->d.be_ny;
    a.be_len = e->d.be_len;
    a.z = e->d.z;
    a.gm2 = e->d.gm2;
    a.area = e->d.area;
    a.inradius = e->d.inr;
    a.bc = e->d.bc;
    a.clock = e->d.clock;
    a.ledger = e->d.ledger;
    a.quiet = e->d.quiet;
    a.run = e->d.run;
    a.act = e->d.act;
    a.store_all = e->params.store_all;
    a.blk_member = e->d.blk_member;
    a.member_end = e->d.member_end;
    a.t_end_m = e->d.t_end;
    a.g = e->params.g;
    a.cfl = e->params.cfl;
    a.h_dry = e->params.h_dry;
    a.dt_max = e->params.dt_max;
    a.t_end = INFINITY;
    a.n_cells = int32_t(e->total_cells);
    const int threads = e->params.block_threads == 0
                            ? e->block_cells
                            : e->params.block_threads;
    a.n_blocks = int32_t(e->total_blocks);
    a.blk_base = 0;
    const swe::StepBuffers b{{e->d.h[0], e->d.h[1]},
                             {e->d.hu[0], e->d.hu[1]},
                             {e->d.hv[0], e->d.hv[1]}};
    hipError_t er = swe::enqueue_steps(
        a, b, e->cur_buf, e->cur_slot, e->step_index, steps,
        swe::StepLaunch{e->block_cells, threads, e->params.load_schedule},
        &e->graph, e->params.graph_steps, e->stream);
    if (er != hipSuccess)
        return efail(e, SWE_EDEVICE,
                     std::string("step launch: ") + hipGetErrorString(er));
    return SWE_OK;
}

swe_status swe_ens_get_time(swe_ens *e, int32_t member, double *t,
                            double *last_dt, int64_t *steps)
{
    if (!e) return SWE_EINVAL;
    if (member < 0 || member >= e->n_members)
        return efail(e, SWE_EINVAL, "member out of range");
    swe_status st = ens_prepare(e);
    if (st) return st;
    Clock ck;
    if ((st = read_member_clock(e, member, &ck))) return st;
    if (t) *t = ck.t[e->cur_slot];
    if (last_dt) *last_dt = ck.last_dt;
    if (steps) *steps = ck.steps;
    return SWE_OK;
}

swe_status swe_ens_get_state(swe_ens *e, int32_t member, double *h,
                             double *hu, double *hv, swe_mem mem)
{
    if (!e) return SWE_EINVAL;
    if (member < 0 || member >= e->n_members)
        return efail(e, SWE_EINVAL, "member out of range");
    if (!h || !hu || !hv) return efail(e, SWE_EINVAL, "null state array");
    if (mem != SWE_MEM_HOST && mem != SWE_MEM_DEVICE)
        return efail(e, SWE_EINVAL, "bad memory kind");
    swe_status st = ens_prepare(e);
    if (st) return st;
    Clock ck;
    if ((st = read_member_clock(e, member, &ck))) return st;
    const size_t n = size_t(e->n_cells[member]);
    const int64_t c0 = e->cell_off[member];
    const int b = e->cur_buf;
    std::vector<double> a(n), bb(n), cc(n);
    ENSCHK(e, hipMemcpyAsync(a.data(), e->d.h[b] + c0, n * 8,
                             hipMemcpyDeviceToHost, e->stream));
    ENSCHK(e, hipMemcpyAsync(bb.data(), e->d.hu[b] + c0, n * 8,
                             hipMemcpyDeviceToHost, e->stream));
    ENSCHK(e, hipMemcpyAsync(cc.data(), e->d.hv[b] + c0, n * 8,
                             hipMemcpyDeviceToHost, e->stream));
    ENSCHK(e, hipStreamSynchronize(e->stream));
    const std::vector<int32_t> &iou = e->internal_of_user[member];
    std::vector<double> x(n), y(n), w(n);
    for (size_t u = 0; u < n; ++u) {
        x[u] = a[iou[u]];
        y[u] = bb[iou[u]];
        w[u] = cc[iou[u]];
    }
    if (mem == SWE_MEM_HOST) {
        std::copy(x.begin(), x.end(), h);
        std::copy(y.begin(), y.end(), hu);
        std::copy(w.begin(), w.end(), hv);
        return SWE_OK;
    }
    ENSCHK(e, hipMemcpyAsync(h, x.data(), n * 8, hipMemcpyHostToDevice,
                             e->stream));
    ENSCHK(e, hipMemcpyAsync(hu, y.data(), n * 8, hipMemcpyHostToDevice,
                             e->stream));
    ENSCHK(e, hipMemcpyAsync(hv, w.data(), n * 8, hipMemcpyHostToDevice,
                             e->stream));
    ENSCHK(e, hipStreamSynchronize(e->stream));
    return SWE_OK;
}

swe_status swe_ens_get_activity(swe_ens *e, int64_t *blocks, int64_t *cells)
{
    if (!e) return SWE_EINVAL;
    swe_status st = ens_prepare(e);
    if (st) return st;
    const int64_t nb = e->total_blocks, B = e->block_cells;
    // the kernel's test: store_all off, the mark of this step's parity
    // clear, and not a member's first block (it advances the clock)
    std::vector<uint32_t> mark(size_t(nb), 1u);
    if (!e->params.store_all) {
        ENSCHK(e, hipMemcpyAsync(mark.data(),
                                 e->d.run + size_t(e->step_index & 1) * nb,
                                 size_t(nb) * 4, hipMemcpyDeviceToHost,
                                 e->stream));
        ENSCHK(e, hipStreamSynchronize(e->stream));
    }
    int64_t b = 0, n = 0;
    for (int64_t k = 0; k < nb; ++k) {
        const int32_t code = e->blk_member[size_t(k)];
        if (!mark[size_t(k)] && code >= 0) continue;
        const int32_t m = code & 0x7fffffff;
        ++b;
        n += std::max<int64_t>(0, std::min<int64_t>(B, e->member_end[m] -
                                                           k * B));
    }
    if (blocks) *blocks = b;
    if (cells) *cells = n;
    return SWE_OK;
}

swe_status swe_ens_info(const swe_ens *e, int64_t *n_cells, int64_t *n_blocks)
{
    if (!e) return SWE_EINVAL;
    int64_t s = 0;
    for (int64_t n : e->n_cells) s += n;
    if (n_cells) *n_cells = s;
    if (n_blocks) *n_blocks = e->total_blocks;
    return SWE_OK;
}

}  // extern "C"
