// HIP kernels (gfx950) of the explicit finite-volume shallow-water step of
// Delmas & Soulaimani (arXiv 2010.14416), sections 2-3.
//
// One launch of swe_step_kernel is one explicit step. A workgroup owns one
// block of consecutive cells in the locality (Hilbert) order:
//   1. it reads the step's time step from the device clock (eq. 15 form
//      computed by the previous step), clipped to t_end;
//   2. it stages its cells' depth, velocity and bed in LDS;
//   3. it evaluates every edge of the block once (hydrostatic
//      reconstruction eq. 28, rotation eq. 12, HLLC eqs. 17-26, bed-slope
//      terms eq. 30, boundary fluxes sec. 3.1) and keeps both sides'
//      contributions in LDS; neighbours in other blocks are read from HBM;
//   4. each thread sums its cell's three contributions in local-side order,
//      applies the semi-implicit Manning update (eqs. 31-37) and the
//      positivity fix, writes U^{n+1} and the cell's R_i / s_i;
//   5. the block's minimum of R_i / s_i (wave shuffles, then LDS) goes to the
//      clock with one 64-bit atomic min on the bit pattern (positive doubles
//      order as unsigned integers), so the next step finds its time step on
//      the device without a host round trip;
//   6. it marks the blocks that must run in the next step: itself unless
//      quiet for two steps, and, across each edge to another block, that
//      block if the cell on this side left the quiet dry path in this step
//      or the block's previous computed one. Unmarked blocks are dormant.
// State and geometry are FP64 structure-of-arrays, read once per step with
// coalesced loads; edges on a block border are evaluated by both blocks.
//
// Arithmetic: every formula is evaluated as written, operation by operation,
// with correctly rounded +, -, *, /, sqrt and no contraction into fused
// multiply-adds, so that results are reproducible bit for bit from the
// formulas (the only library function is cbrt, in the friction coefficient).
#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

#include <cfloat>
#include <climits>
#include <cmath>

#include "swe_device.hpp"
#include "swe_mesh.hpp"
#include "swe_scheme.hpp"

namespace swe {
namespace {

constexpr unsigned long long kInfBits = 0x7ff0000000000000ull;

__device__ __forceinline__ CellState load_cell(const StepArgs &a, int c)
{
    CellState s;
    s.h = at(a.h0, c);
    const double hu = at(a.hu0, c), hv = at(a.hv0, c);
    s.z = at(a.z, c);
    if (s.h > a.h_dry) {
        const double r = 1.0 / s.h;
        s.u = hu * r;
        s.v = hv * r;
    } else {
        s.u = 0.0;
        s.v = 0.0;
    }
    return s;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// End of a step for one block: wave-shuffle then LDS reductions of the
// block's min R_i/s_i (one 64-bit atomic min into the next clock slot), of
// the mass added by the positivity fix, and of the non-finite flag; block 0
// advances the clock. Each wave of owned cells records which of them left
// the quiet dry path (act_now and a.act). Returns the block's new count of
// consecutive quiet steps (capped at 2) to every thread.
template <int NC, int NT>
__device__ __forceinline__ int block_finish(const StepArgs &a, int blk,
                                             Clock *clock, bool first,
                                             double rs, double clamp,
                                             unsigned bad, bool active,
                                             int quiet_steps, bool unbounded,
                                             double dt, double tn,
                                             long long idx, int nxt,
                                             double *red_min, double *red_sum,
                                             unsigned *red_bad,
                                             unsigned long long *act_now)
{
    const int tid = threadIdx.x;
    rs = wave_min(rs);
    clamp = wave_sum(clamp);
    const unsigned long long ballot = __ballot(bad != 0u);
    const unsigned long long busy = __ballot(active);
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0) {
        red_min[wave] = rs;
        red_sum[wave] = clamp;
        red_bad[wave] = (ballot != 0ull ? 1u : 0u) | (busy != 0ull ? 2u : 0u);
        if (wave < NC / 64) {
            act_now[wave] = busy;
            a.act[size_t(blk) * (NC / 64) + wave] = busy;
        }
    }
    __syncthreads();
    unsigned busy_any = 0u;
    for (int w = 0; w < NT / 64; ++w) busy_any |= red_bad[w] & 2u;
    const int q = busy_any ? 0 : min(quiet_steps + 1, 2);
    if (tid == 0) {
        double m = red_min[0], cs = red_sum[0];
        unsigned flags = red_bad[0];
        for (int w = 1; w < NT / 64; ++w) {
            m = fmin(m, red_min[w]);
            cs += red_sum[w];
            flags |= red_bad[w];
        }
        const bool anybad = (flags & 1u) != 0u;
        if (q != quiet_steps) a.quiet[blk] = q;
        if (m < INFINITY)
            atomicMin(&clock->minrs[nxt][blockIdx.x & (kClockLanes - 1)][0],
                      (unsigned long long)__double_as_longlong(m));
        if (cs != 0.0) a.ledger[blk] += cs;
        if (anybad || unbounded) {
            atomicOr(&clock->health, (anybad ? 1u : 0u) | (unbounded ? 2u : 0u));
            atomicMin(&clock->bad_step, idx);
        }
        if (first) {
            const int nn = nxt == 2 ? 0 : nxt + 1;
            clock->t[nxt] = tn;
            clock->idx[nxt] = idx + 1;
            clock->dt_ring[idx & 7] = dt;
            // the empty steps launched after t_end leave the last time
            // step and the step count alone
            if (dt > 0.0) {
                clock->last_dt = dt;
                clock->steps += 1;
            }
            for (int x = 0; x < kClockLanes; ++x)
                atomicExch(&clock->minrs[nn][x][0], kInfBits);
        }
    }
    return q;
}

// Clock words of this step, read with one vector load per lane so that they
// travel with the block's first loads: lane x < kClockLanes holds lane x of
// the time-step minimum, lane kClockLanes the time t, lane kClockLanes + 1
// the step index.
__device__ __forceinline__ double clock_word(const StepArgs &a,
                                             const Clock *c)
{
    const int lane = int(threadIdx.x & 63u);
    if (lane < kClockLanes)
        return __longlong_as_double((long long)c->minrs[a.cur][lane][0]);
    if (lane == kClockLanes) return c->t[a.cur];
    if (lane == kClockLanes + 1) return __longlong_as_double(c->idx[a.cur]);
    return 0.0;
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(b), lane));
    const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(b >> 32), lane));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// v from the lane that the DPP control CTRL selects within each row of 16
// (0 where there is none); the lanes of the wave are all active.
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo =
        unsigned(__builtin_amdgcn_mov_dpp(int(b), CTRL, 0xf, 0xf, true));
    const unsigned hi =
        unsigned(__builtin_amdgcn_mov_dpp(int(b >> 32), CTRL, 0xf, 0xf, true));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ StepTime step_time(const StepArgs &a, double word,
                                              double t_end)
{
    static_assert(kClockLanes == 8, "the lane minimum combines 8 lanes");
    StepTime st;
    // minimum of lanes 0..7 into lane 0 in vector registers: swap neighbours
    // (quad_perm 1,0,3,2), then pairs (quad_perm 2,3,0,1), then lane 4 into
    // lane 0 (row_shl 4); the minimum of non-negative words takes no order
    double m = fmin(word, dpp_double<0xB1>(word));
    m = fmin(m, dpp_double<0x4E>(m));
    m = fmin(m, dpp_double<0x104>(m));
    const double mrs = read_lane(m, 0);
    const double t = read_lane(word, kClockLanes);
    st.idx = __double_as_longlong(read_lane(word, kClockLanes + 1));
    st.dt = fmin(a.cfl * mrs, a.dt_max);
    const double rem = t_end - t;
    if (st.dt >= rem) {
        st.dt = rem > 0.0 ? rem : 0.0;
        st.tn = rem > 0.0 ? t_end : t;
    } else {
        st.tn = t + st.dt;
    }
    st.unbounded = !(st.dt < INFINITY);
    if (st.unbounded) {
        st.dt = 0.0;
        st.tn = t;
    }
    return st;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2. Workgroup w runs block xcd_block(w): runs of kXcdChunk consecutive
// blocks (neighbours along the space-filling curve, which share halo cells)
// go to one XCD, and the runs are dealt round-robin so that every XCD gets
// a similar mix of wet and dry blocks. Blocks past the last whole round of
// 8 kXcdChunk keep their own index.
constexpr int kXcdChunk = 4;

__device__ __forceinline__ int xcd_block(int w, int n_blocks)
{
    constexpr int R = 8 * kXcdChunk;
    if (w >= (n_blocks / R) * R) return w;
    const int x = w & 7, j = w >> 3;
    return (j / kXcdChunk) * R + x * kXcdChunk + j % kXcdChunk;
}

// An edge record (va, vb) that joins a cell of this block to a cell x of
// another: the first cell of x's block plus the local index of this
// block's cell (below 2^30); else all ones.
template <int NC>
__device__ __forceinline__ uint32_t cross_mark(int32_t va, int32_t vb)
{
    const bool xa = uint32_t(va) < kSideBoundary;
    const bool xb = uint32_t(vb) < kSideBoundary;
    if (!xa && !xb) return 0xffffffffu;
    return (uint32_t(xa ? va : vb) & ~uint32_t(NC - 1)) |
           (uint32_t(xa ? vb : va) & uint32_t(NC - 1));
}

// One explicit step, one workgroup per block of NC consecutive cells and NT
// threads (NC or 2 NC); threads below NC own a cell, all threads share the
// block's edges (neighbour-block and boundary edges first, so that the
// first NT of them hold every edge that needs a neighbour's state).
//
// Before the first barrier each thread requests its owned cell and its
// edge records, then, in one second round trip, the state of its first
// edge's neighbour in another block and its cell's momentum if wet; the
// cell geometry of wet cells is requested before the second barrier.
// EAGER: the geometry of every edge and cell is requested with them.
// Otherwise inputs that cannot change the result are skipped: the geometry
// of an edge between two cells holding no water is never read, and a dry
// cell reads its area and inscribed radius only if it receives flux.
// Both read the same values and round identically.
// SLOT: the output is a fresh slot (the adjoint's stored states): every cell
// stores, a dormant block copies its state over, and which blocks ran is
// recorded in a.run_log (if not null). A separate instantiation, so that
// the plain step keeps its registers.
template <int NC, int NT, bool EAGER, bool MON, bool SLOT>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(6)))
void swe_step_kernel(StepArgs a)
{
    extern __shared__ double lds[];
    __shared__ double red_min[NT / 64];
    __shared__ double red_sum[NT / 64];
    __shared__ unsigned red_bad[NT / 64];
    __shared__ int4 s_bnd[1];
    // per wave of owned cells: those not quiet in the block's last
    // computed step, then those not quiet in this one
    __shared__ unsigned long long s_act[2 * (NC / 64)];
    double *s_h = lds;
    double *s_u = s_h + NC;
    double *s_v = s_u + NC;
    double *s_z = s_v + NC;
    double *s_c = s_z + NC;   // [3 components][3 sides][NC cells]

    const int tid = threadIdx.x;
    const int blk = a.blk_base + xcd_block(blockIdx.x, a.n_blocks);
    const int c0 = blk * NC;
    // run marks of this step's parity
    const size_t run_at = size_t(a.step_index & 1) * size_t(a.n_blocks);
    const uint32_t run_me = a.run[run_at + blk];
    // one mesh, or member `mem` of an ensemble (its cells start on a block)
    int mem = 0, cell_end = a.n_cells;
    bool first = blk == 0;
    if (a.blk_member) {
        const int code = a.blk_member[blk];
        first = code < 0;
        mem = code & 0x7fffffff;
        cell_end = a.member_end[mem];
    }
    // dormant blocks: a block whose cells took the quiet dry path in the two
    // previous steps, as did every cell of another block that shares an
    // edge with them, has the inputs it had one step ago, so it would
    // compute (and already holds) the same quiet results. No block of the
    // previous step marked it to run: it returns before any other load
    // (the clock's block always runs).
    if (!a.store_all && !first && run_me == 0u) {
        if (SLOT && a.run_log && tid == 0) a.run_log[blk] = 0;
        if (SLOT && tid < NC && blk * NC + tid < cell_end) {
            // a fresh output slot: carry the unchanged state over
            const int c = blk * NC + tid;
            at(a.h1, c) = at(a.h0, c);
            at(a.hu1, c) = at(a.hu0, c);
            at(a.hv1, c) = at(a.hv0, c);
            if (a.r_out) {
                a.r_out[c] = 0.0;
                a.r_out[a.n_cells + c] = 0.0;
                a.r_out[2 * a.n_cells + c] = 0.0;
            }
        }
        return;
    }
    Clock *clock = a.clock + mem;
    const double t_end = a.t_end_m ? a.t_end_m[mem] : a.t_end;
    const int nc = min(NC, cell_end - c0);
    // an ensemble pads every member to whole blocks, so the block's NC
    // cells can be read before the member's cell count has arrived
    const int nc_read = a.blk_member ? NC : min(NC, a.n_cells - c0);
    const int e0 = a.blk_edge[blk];
    const int ne = a.blk_edge[blk + 1] - e0;
    const bool owner = tid < NC && tid < nc;
    const int i = c0 + tid;
    const double g = a.g, h_dry = a.h_dry;

    // phase 1: owned cell, first edge record (+ geometry), neighbour state
    const int quiet_steps = a.quiet[blk];
    // the block's boundary slots (discharge monitors), to LDS with phase 1
    int4 bnd = make_int4(0, 0, 0, 0);
    if (MON && tid == NC / 64)
        bnd = *reinterpret_cast<const int4 *>(a.mon->blk_bnd + 4 * blk);
    double h = 0.0, hu = 0.0, hv = 0.0, zc = 0.0;
    if (tid < NC && tid < nc_read) {
        h = at(a.h0, i);
        zc = at(a.z, i);
    }
    const double cw = clock_word(a, clock);
    int32_t ea = 0, eb = 0, ea2 = 0, eb2 = 0;
    double nx = 0.0, ny = 0.0, len = 0.0;
    if (tid < ne) {
        ea = at(a.be_a, e0 + tid);
        eb = at(a.be_b, e0 + tid);
        if (EAGER) {
            nx = at(a.be_nx + e0, tid);
            ny = at(a.be_ny + e0, tid);
            len = at(a.be_len + e0, tid);
        }
    }
    if (tid + NT < ne) {              // the thread's second edge record
        ea2 = at(a.be_a, e0 + tid + NT);
        eb2 = at(a.be_b, e0 + tid + NT);
    }
    unsigned long long act_prev = 0ull;   // to s_act with phase 1
    if (tid < NC && (tid & 63) == 0)
        act_prev = a.act[size_t(blk) * (NC / 64) + (tid >> 6)];
    // a side coded as a plain internal index (below kSideBoundary) is a
    // cell of another block
    CellState X;
    // the thread's first and second edge records, if they join a cell of
    // this block to one of another (cross_mark), for the run marks
    uint32_t xmark = 0xffffffffu, xmark2 = 0xffffffffu;
    {
        double xh = 0.0, xhu = 0.0, xhv = 0.0, xz = 0.0;
        const bool xa = uint32_t(ea) < kSideBoundary;
        const bool xb = uint32_t(eb) < kSideBoundary;
        if (tid < ne && (xa || xb)) {
            const int x = xa ? ea : eb;
            xmark = cross_mark<NC>(ea, eb);
            xh = at(a.h0, x);
            xhu = at(a.hu0, x);
            xhv = at(a.hv0, x);
            xz = at(a.z, x);
        }
        // the momentum of a dry cell is read in phase 3, and only if needed
        // (requested after the neighbour state, whose address arrived first)
        if (owner && h > h_dry) {
            hu = at(a.hu0, i);
            hv = at(a.hv0, i);
        }
        X.h = xh;
        X.z = xz;
        X.u = 0.0;
        X.v = 0.0;
        if (xh > h_dry) {
            const double r = 1.0 / xh;
            X.u = xhu * r;
            X.v = xhv * r;
        }
    }
    const StepTime st = step_time(a, cw, t_end);
    if (MON && tid == NC / 64) s_bnd[0] = bnd;
    if (tid < NC && (tid & 63) == 0) s_act[tid >> 6] = act_prev;
    if (owner) {
        s_h[tid] = h;
        s_z[tid] = zc;
        if (h > h_dry) {
            const double r = 1.0 / h;
            s_u[tid] = hu * r;
            s_v[tid] = hv * r;
        } else {
            s_u[tid] = 0.0;
            s_v[tid] = 0.0;
        }
    }
    __syncthreads();

    // phase 2: every edge of the block once. Contributions go straight into
    // the LDS slots [component][side][cell] of the one or two cells of the
    // block the edge bounds. An edge between two cells holding no water
    // (h == 0), or a wall / transmissive edge of such a cell, adds exact
    // zeros.
    // one edge: its record (va, vb), the state Y of a side in another
    // block, the geometry (if already loaded)
    auto edge = [&](int k, int32_t va, int32_t vb, const CellState &Y,
                    double enx, double eny, double elen) {
        const Side pa = decode_side(va), pb = decode_side(vb);
        CellState Lc, Rc;
        Rc.h = 0.0; Rc.u = 0.0; Rc.v = 0.0; Rc.z = 0.0;
        if (pa.kind == 0) {
            Lc.h = s_h[pa.local]; Lc.u = s_u[pa.local];
            Lc.v = s_v[pa.local]; Lc.z = s_z[pa.local];
        } else {
            Lc = Y;
        }
        bool idle;
        BcEntry bc{};
        if (pb.kind == 2) {
            bc = a.bc[pb.global];
            idle = Lc.h == 0.0 && (bc.kind == 0 || bc.kind == 1);
        } else {
            if (pb.kind == 0) {
                Rc.h = s_h[pb.local]; Rc.u = s_u[pb.local];
                Rc.v = s_v[pb.local]; Rc.z = s_z[pb.local];
            } else {
                Rc = Y;
            }
            idle = Lc.h == 0.0 && Rc.h == 0.0;
        }
        double cl0 = 0.0, cl1 = 0.0, cl2 = 0.0;
        double cr0 = 0.0, cr1 = 0.0, cr2 = 0.0;
        if (!idle) {
            if (!EAGER) {
                enx = at(a.be_nx + e0, k);
                eny = at(a.be_ny + e0, k);
                elen = at(a.be_len + e0, k);
            }
            edge_contrib(g, h_dry, pb.kind == 2, bc, Lc, Rc, enx, eny, elen,
                         cl0, cl1, cl2, cr0, cr1, cr2);
        }

        if (pa.kind == 0) {
            double *d = s_c + pa.k * NC + pa.local;
            d[0] = cl0;
            d[3 * NC] = cl1;
            d[6 * NC] = cl2;
        }
        if (pb.kind == 0) {
            double *d = s_c + pb.k * NC + pb.local;
            d[0] = cr0;
            d[3 * NC] = cr1;
            d[6 * NC] = cr2;
        }
    };
    if (tid < ne) edge(tid, ea, eb, X, nx, ny, len);
    for (int k = tid + NT; k < ne; k += NT) {   // blocks with > NT edges
        int32_t va = ea2, vb = eb2;
        if (k != tid + NT) {
            va = at(a.be_a, e0 + k);
            vb = at(a.be_b, e0 + k);
        } else {
            xmark2 = cross_mark<NC>(va, vb);
        }
        double enx = 0.0, eny = 0.0, elen = 0.0;
        if (EAGER) {
            enx = at(a.be_nx + e0, k);
            eny = at(a.be_ny + e0, k);
            elen = at(a.be_len + e0, k);
        }
        CellState Y;
        Y.h = 0.0; Y.u = 0.0; Y.v = 0.0; Y.z = 0.0;
        if (uint32_t(va) < kSideBoundary) Y = load_cell(a, va);
        if (uint32_t(vb) < kSideBoundary) Y = load_cell(a, vb);
        edge(k, va, vb, Y, enx, eny, elen);
    }
    // cell geometry: every cell (EAGER), else the wet ones, which always
    // need it; a dry cell requests its own in phase 3 if it receives flux
    double area = 0.0, gm2 = 0.0, inr = 0.0;
    const double hc = owner ? s_h[tid] : 0.0;   // h of the owned cell
    if (owner && (EAGER || hc > h_dry)) {
        area = at(a.area, i);
        gm2 = at(a.gm2, i);
        inr = at(a.inradius, i);
    }
    __syncthreads();

    // phase 3: each owned cell sums its three sides in side order, updates
    // and writes U^{n+1}; R_i/s_i, the clamped mass and the non-finite flag
    // go to the block reduction. A dry cell whose three sides bring exact
    // zeros needs no area (R/A = R exactly).
    double rs = INFINITY, clamp = 0.0;
    unsigned bad = 0;
    bool active = owner;   // owned cell not on the quiet dry path
    double hn = hc, hun = 0.0, hvn = 0.0;   // U^{n+1} of the owned cell
    if (owner) {
        double R0 = 0.0, R1 = 0.0, R2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            R0 += s_c[k * NC + tid];
            R1 += s_c[(3 + k) * NC + tid];
            R2 += s_c[(6 + k) * NC + tid];
        }
        if (SLOT && a.r_out) {
            a.r_out[i] = R0;
            a.r_out[a.n_cells + i] = R1;
            a.r_out[2 * a.n_cells + i] = R2;
        }
        hun = hu;
        hvn = hv;
        const double dt = st.dt;
        if (dt > 0.0 && hc <= h_dry && R0 == 0.0 && R1 == 0.0 && R2 == 0.0) {
            // no friction below h_dry; h + dt*(+-0) cannot go negative
            hn = hc + dt * R0;
            hun = 0.0;
            hvn = 0.0;
            active = false;
        } else {
            if (hc <= h_dry) {
                hu = at(a.hu0, i);
                hv = at(a.hv0, i);
                if (!EAGER) {
                    area = at(a.area, i);
                    inr = at(a.inradius, i);
                }
            }
            hun = hu;
            hvn = hv;
            if (dt > 0.0)
                cell_update(h_dry, dt, area, hc > h_dry ? gm2 : 0.0, hc, hu,
                            hv, R0, R1, R2, hn, hun, hvn, clamp);
        }
        if (!isfinite(hn) || !isfinite(hun) || !isfinite(hvn)) bad = 1u;
        if (hn > h_dry) {
            const double r = 1.0 / hn;
            const double u = hun * r, v = hvn * r;
            rs = inr / (sqrt(g * hn) + sqrt(u * u + v * v));
        }
    }
    const int q = block_finish<NC, NT>(a, blk, clock, first, rs, clamp, bad,
                                   active, quiet_steps, st.unbounded, st.dt,
                                   st.tn, st.idx, a.cur == 2 ? 0 : a.cur + 1,
                                   red_min,
                                   red_sum, red_bad, s_act + NC / 64);
    {
        // this step's mark is used up; a block not quiet for two steps
        // marks itself to run at the next step, and each edge from a cell
        // that may have changed marks the other block it reaches
        const size_t next = size_t(a.n_blocks) - run_at;
        if (tid == 0 && run_me) a.run[run_at + blk] = 0u;
        if (SLOT && tid == 0 && a.run_log) a.run_log[blk] = 1;
        if (q < 2) {
            if (tid == 0) a.run[next + blk] = 1u;
            // a cell may have changed in this step if it was not quiet in
            // it or in the block's last computed step (a cell quiet in both
            // holds (h, 0, 0) before and after)
            auto mark = [&](uint32_t m) {
                const uint32_t l = m & uint32_t(NC - 1);
                const unsigned long long w =
                    s_act[l >> 6] | s_act[NC / 64 + (l >> 6)];
                if (m != 0xffffffffu && (w >> (l & 63)) & 1ull)
                    a.run[next + m / NC] = 1u;
            };
            mark(xmark);
            mark(xmark2);
            // records to other blocks come first: past the thread's second
            // record only if that one reaches another block
            for (int k = tid + 2 * NT; xmark2 != 0xffffffffu && k < ne;
                 k += NT) {
                const uint32_t m =
                    cross_mark<NC>(at(a.be_a, e0 + k), at(a.be_b, e0 + k));
                if (m == 0xffffffffu) break;
                mark(m);
            }
        }
    }
    // the stores come last: no instruction after them waits for a load, so
    // the wave never waits for its own stores. A quiet cell of a block quiet
    // in the two previous steps already holds (h, 0, 0) in the output buffer
    // (it held U^{n-1} = U^n).
    if (owner && (active || quiet_steps < 2 || a.store_all || SLOT)) {
        at(a.h1, i) = hn;
        at(a.hu1, i) = hun;
        at(a.hv1, i) = hvn;
    }
    if (MON && owner && hn > hc) {
        // flood envelope: h_max >= h always holds, so the highest depth can
        // only change where the depth rose
        const double hm = a.mon->h_max[i];
        if (hn > hm) {
            a.mon->h_max[i] = hn;
            if (hm <= h_dry && hn > h_dry) a.mon->t_wet[i] = st.tn;
        }
    }
    if (MON && s_bnd[0].z > 0) {
        // discharge monitors of the block's boundary slots: the volume
        // leaving per unit time, L G_1 = -(the edge's mass contribution to
        // its cell), read back from the cell's side slot. One edge per
        // slot: the volume's single addition is the plain sum (an atomic
        // only so that nothing waits for it).
        const int4 b = s_bnd[0];
        for (int k = tid; k < b.z; k += NT) {
            const Side pa = decode_side(at(a.be_a, b.y + k));
            const double rate = -s_c[pa.k * NC + pa.local];
            a.mon->mon_rate[b.x + k] = rate;
            unsafeAtomicAdd(&a.mon->mon_vol[b.x + k], st.dt * rate);
        }
    }
}

__global__ void clock_set_kernel(Clock *c, double t, long long steps,
                                 long long step_index)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->t[0] = t;
        c->t[1] = t;
        c->t[2] = t;
        c->idx[0] = step_index;
        c->idx[1] = step_index;
        c->idx[2] = step_index;
        for (int s = 0; s < 3; ++s)
            for (int x = 0; x < kClockLanes; ++x) c->minrs[s][x][0] = kInfBits;
        c->last_dt = 0.0;
        c->steps = steps;
        c->health = 0u;
        c->pad = 0u;
        c->bad_step = LLONG_MAX;
    }
}

__global__ void slot_reset_kernel(Clock *c, int slot)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        for (int x = 0; x < kClockLanes; ++x)
            atomicExch(&c->minrs[slot][x][0], kInfBits);
}

__global__ __launch_bounds__(256) void min_rs_kernel(
    const double *__restrict__ h, const double *__restrict__ hu,
    const double *__restrict__ hv, const double *__restrict__ inr, int64_t n,
    double g, double h_dry, Clock *c, int cur)
{
    __shared__ double red[4];
    double rs = INFINITY;
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x) {
        const double hk = h[k];
        if (hk > h_dry) {
            const double r = 1.0 / hk;
            const double u = hu[k] * r, v = hv[k] * r;
            rs = fmin(rs, inr[k] / (sqrt(g * hk) + sqrt(u * u + v * v)));
        }
    }
    rs = wave_min(rs);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rs;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
        if (m < INFINITY)
            atomicMin(&c->minrs[cur][blockIdx.x & (kClockLanes - 1)][0],
                      (unsigned long long)__double_as_longlong(m));
    }
}

__global__ __launch_bounds__(256) void gather3_kernel(
    const double *__restrict__ a, const double *__restrict__ b,
    const double *__restrict__ c, double *__restrict__ A,
    double *__restrict__ B, double *__restrict__ C,
    const int32_t *__restrict__ idx, int64_t n)
{
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x) {
        const int64_t j = idx[k];
        A[k] = a[j];
        B[k] = b[j];
        C[k] = c[j];
    }
}

__global__ __launch_bounds__(256) void gather1_kernel(
    const double *__restrict__ a, double *__restrict__ A,
    const int32_t *__restrict__ idx, int64_t n)
{
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x)
        A[k] = a[idx[k]];
}

__global__ __launch_bounds__(256) void check_state_kernel(
    const double *__restrict__ h, const double *__restrict__ hu,
    const double *__restrict__ hv, int64_t n, unsigned *flag)
{
    bool bad = false;
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x) {
        const double hk = h[k];
        if (!(hk >= 0.0) || !isfinite(hk) || !isfinite(hu[k]) ||
            !isfinite(hv[k]))
            bad = true;
    }
    if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

__global__ __launch_bounds__(256) void check_field_kernel(
    const double *__restrict__ f, int64_t n, int nonneg, unsigned *flag)
{
    bool bad = false;
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x) {
        const double v = f[k];
        if (!isfinite(v) || (nonneg && !(v >= 0.0))) bad = true;
    }
    if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

__global__ __launch_bounds__(256) void gm2_kernel(
    const double *__restrict__ m, double *__restrict__ gm2, int64_t n,
    double g)
{
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x)
        gm2[k] = g * m[k] * m[k];
}

// Per-part partial sums of |Omega_i| h_i and of wet cells; part p covers a
// fixed contiguous range, summed in a fixed order, so the result does not
// depend on scheduling.
__global__ __launch_bounds__(kDiagThreads) void diag_kernel(
    const double *__restrict__ h, const double *__restrict__ area, int64_t n,
    double h_dry, double *part_mass, unsigned long long *part_wet)
{
    __shared__ double sm[kDiagThreads / 64];
    __shared__ unsigned long long sw[kDiagThreads / 64];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t k0 = int64_t(blockIdx.x) * per;
    const int64_t k1 = min(n, k0 + per);
    double m = 0.0;
    unsigned long long w = 0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
        m += area[k] * h[k];
        w += h[k] > h_dry ? 1ull : 0ull;
    }
    m = wave_sum(m);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
    if ((threadIdx.x & 63) == 0) {
        sm[threadIdx.x >> 6] = m;
        sw[threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        unsigned long long c = 0;
        for (int q = 0; q < kDiagThreads / 64; ++q) {
            s += sm[q];
            c += sw[q];
        }
        part_mass[blockIdx.x] = s;
        part_wet[blockIdx.x] = c;
    }
}

__global__ __launch_bounds__(256) void fill_u32_kernel(unsigned *p,
                                                       unsigned v, int64_t n)
{
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x)
        p[k] = v;
}

__global__ __launch_bounds__(256) void fill_f64_kernel(double *p, double v,
                                                       int64_t n)
{
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x)
        p[k] = v;
}

__global__ __launch_bounds__(256) void envelope_reset_kernel(
    const double *h, int64_t n, double h_dry, double t, double *h_max,
    double *t_wet)
{
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x) {
        h_max[k] = h[k];
        t_wet[k] = h[k] > h_dry ? t : INFINITY;
    }
}

inline unsigned grid_for(int64_t n, int threads = 256)
{
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return unsigned(b);
}

}  // namespace

size_t step_lds_bytes(int block_cells)
{
    return sizeof(double) * 13 * size_t(block_cells);
}

namespace {
template <int NC, int NT, bool MON, bool SLOT>
void launch_mon(const StepArgs &a, int schedule, hipStream_t s)
{
    if (schedule == 0)
        hipLaunchKernelGGL((swe_step_kernel<NC, NT, false, MON, SLOT>),
                           dim3(a.n_blocks), dim3(NT), step_lds_bytes(NC), s,
                           a);
    else
        hipLaunchKernelGGL((swe_step_kernel<NC, NT, true, MON, SLOT>),
                           dim3(a.n_blocks), dim3(NT), step_lds_bytes(NC), s,
                           a);
}

template <int NC, int NT, bool SLOT>
void launch_slot(const StepArgs &a, int schedule, hipStream_t s)
{
    if (a.mon)
        launch_mon<NC, NT, true, SLOT>(a, schedule, s);
    else
        launch_mon<NC, NT, false, SLOT>(a, schedule, s);
}

// Steps into fresh slots (the adjoint's) exist for 256-cell blocks only.
template <int NC, int NT>
hipError_t launch_one(const StepArgs &a, int schedule, hipStream_t s)
{
    if (!a.fresh_out) {
        launch_slot<NC, NT, false>(a, schedule, s);
        return hipSuccess;
    }
    if constexpr (NC == 256) {
        launch_slot<NC, NT, true>(a, schedule, s);
        return hipSuccess;
    }
    return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_step(const StepArgs &a, int block_cells, int threads,
                       int schedule, hipStream_t s)
{
    const bool twice = threads == 2 * block_cells;
    if (!twice && threads != block_cells) return hipErrorInvalidValue;
    hipError_t e;
    switch (block_cells) {
    case 64:
        e = twice ? launch_one<64, 128>(a, schedule, s)
                  : launch_one<64, 64>(a, schedule, s);
        break;
    case 128:
        e = twice ? launch_one<128, 256>(a, schedule, s)
                  : launch_one<128, 128>(a, schedule, s);
        break;
    case 256:
        e = twice ? launch_one<256, 512>(a, schedule, s)
                  : launch_one<256, 256>(a, schedule, s);
        break;
    case 512:
        e = twice ? launch_one<512, 1024>(a, schedule, s)
                  : launch_one<512, 512>(a, schedule, s);
        break;
    default:
        return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_clock_set(Clock *c, double t, long long steps,
                            long long step_index, hipStream_t s)
{
    hipLaunchKernelGGL(clock_set_kernel, dim3(1), dim3(64), 0, s, c, t, steps,
                       step_index);
    return hipGetLastError();
}

hipError_t launch_slot_reset(Clock *c, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(slot_reset_kernel, dim3(1), dim3(64), 0, s, c, slot);
    return hipGetLastError();
}

hipError_t launch_min_rs(const double *h, const double *hu, const double *hv,
                         const double *inr, int64_t n, double g, double h_dry,
                         Clock *c, int cur, hipStream_t s)
{
    hipLaunchKernelGGL(min_rs_kernel, dim3(grid_for(n)), dim3(256), 0, s, h,
                       hu, hv, inr, n, g, h_dry, c, cur);
    return hipGetLastError();
}

hipError_t launch_gather3(const double *a, const double *b, const double *c,
                          double *A, double *B, double *C, const int32_t *idx,
                          int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(gather3_kernel, dim3(grid_for(n)), dim3(256), 0, s, a,
                       b, c, A, B, C, idx, n);
    return hipGetLastError();
}

hipError_t launch_gather1(const double *a, double *A, const int32_t *idx,
                          int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(gather1_kernel, dim3(grid_for(n)), dim3(256), 0, s, a,
                       A, idx, n);
    return hipGetLastError();
}

hipError_t launch_check_state(const double *h, const double *hu,
                              const double *hv, int64_t n, unsigned *flag,
                              hipStream_t s)
{
    hipLaunchKernelGGL(check_state_kernel, dim3(grid_for(n)), dim3(256), 0, s,
                       h, hu, hv, n, flag);
    return hipGetLastError();
}

hipError_t launch_check_field(const double *f, int64_t n, int nonneg,
                              unsigned *flag, hipStream_t s)
{
    hipLaunchKernelGGL(check_field_kernel, dim3(grid_for(n)), dim3(256), 0, s,
                       f, n, nonneg, flag);
    return hipGetLastError();
}

hipError_t launch_gm2(const double *m, double *gm2, int64_t n, double g,
                      hipStream_t s)
{
    hipLaunchKernelGGL(gm2_kernel, dim3(grid_for(n)), dim3(256), 0, s, m, gm2,
                       n, g);
    return hipGetLastError();
}

hipError_t launch_diag(const double *h, const double *area, int64_t n,
                       double h_dry, double *part_mass,
                       unsigned long long *part_wet, int nparts, hipStream_t s)
{
    hipLaunchKernelGGL(diag_kernel, dim3(nparts), dim3(kDiagThreads), 0, s, h,
                       area, n, h_dry, part_mass, part_wet);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, unsigned v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p,
                       v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, p,
                       v, n);
    return hipGetLastError();
}

hipError_t launch_envelope_reset(const double *h, int64_t n, double h_dry,
                                 double t, double *h_max, double *t_wet,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(envelope_reset_kernel, dim3(grid_for(n)), dim3(256), 0,
                       s, h, n, h_dry, t, h_max, t_wet);
    return hipGetLastError();
}

}  // namespace swe
