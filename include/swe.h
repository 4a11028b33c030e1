/*
 * swe.h -- C interface of the explicit finite-volume shallow-water step on
 * unstructured triangles for AMD Instinct MI355X (gfx950).
 *
 * Method: Delmas & Soulaimani, "Multi-GPU implementation of a time-explicit
 * finite volume solver for the Shallow-Water Equations using CUDA and a
 * CUDA-Aware version of OpenMPI", arXiv 2010.14416. The conserved state is
 * U = (h, hu, hv) per triangle (eq. 1, cell averages of eq. 7); each step
 * evaluates the HLLC flux of every edge on hydrostatically reconstructed
 * states (sec. 3.2, eqs. 17-26 and 28), the bed-slope term (eq. 30), the
 * semi-implicit Manning friction (eqs. 31-36), the explicit update (eq. 37)
 * and the CFL time step (eq. 15 with the inscribed radius, sec. 3.1), all on
 * the device.
 *
 * Conventions
 *  - Every call returns a swe_status; swe_last_error() gives a message. No
 *    exception crosses the interface.
 *  - Input pointers are caller-owned and copied during the call; nothing is
 *    retained. Outputs are written into caller-allocated arrays.
 *  - Per-cell arrays follow the caller's triangle order ("user order"). The
 *    library reorders cells internally for locality; that order is invisible
 *    except through swe_get_cell_order().
 *  - SI units. Node and cell indices are 0-based int32.
 *  - A context is not thread-safe; several contexts may coexist.
 *  - Host-side validation (mesh, fields, state, parameters) needs no GPU;
 *    device memory is set up on first use (swe_advance, swe_get_state,
 *    device-pointer inputs, swe_get_diagnostics).
 */
#ifndef SWE_H
#define SWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWE_ABI_VERSION 1
#define SWE_MAX_TAG 1024

typedef struct swe_ctx swe_ctx;

typedef enum {
    SWE_OK = 0,
    SWE_EINVAL = -1,     /* bad argument (null pointer, size, parameter)   */
    SWE_EMESH = -2,      /* invalid mesh (degenerate, non-manifold, ...)    */
    SWE_ESTATE = -3,     /* invalid field or state (NaN, h < 0, n < 0)      */
    SWE_EDEVICE = -4,    /* HIP runtime error or no usable device           */
    SWE_ENOMEM = -5,     /* host or device allocation failed / workspace    */
    SWE_ENOTREADY = -6,  /* call out of order (e.g. no mesh yet)            */
    SWE_ENUMERIC = -7    /* non-finite state or unbounded time step         */
} swe_status;

/* Boundary-condition kinds (sec. 3.1). WALL, TRANSMISSIVE and INFLOW are
 * the paper's three kinds; FIXED_DEPTH and FIXED_STAGE hold a downstream
 * water level and are additions (a ghost state of the given depth, or of
 * depth max(0, stage - z_i), with the cell's velocity, through HLLC). */
typedef enum {
    SWE_BC_WALL = 0,          /* value ignored                                */
    SWE_BC_TRANSMISSIVE = 1,  /* value ignored                                */
    SWE_BC_INFLOW = 2,        /* value = total discharge Q of the tag [m^3/s],
                                 spread uniformly over the tag's edge length */
    SWE_BC_FIXED_DEPTH = 3,   /* value = ghost depth [m], >= 0                */
    SWE_BC_FIXED_STAGE = 4    /* value = ghost water-surface elevation [m]    */
} swe_bc_kind;

typedef enum { SWE_MEM_HOST = 0, SWE_MEM_DEVICE = 1 } swe_mem;

typedef struct {
    double g;              /* gravity [m/s^2] > 0 (9.81)                       */
    double cfl;            /* CFL number of eq. 15, > 0 (0.9, sec. 3.1)        */
    double h_dry;          /* wet/dry depth threshold [m] >= 0 (1e-6)          */
    double dt_max;         /* upper bound on the time step [s] > 0 (+inf)      */
    int32_t check_every;   /* steps between host polls of the device clock
                              when t_end is finite (64)                       */
    int32_t block_cells;   /* cells per mesh block: 64, 128, 256 or 512
                              (256); takes effect at the next set_mesh       */
    int32_t reorder;       /* 1: space-filling-curve cell order (default);
                              0: keep the user order; next set_mesh           */
    int32_t block_threads; /* threads per block: block_cells, 2*block_cells,
                              or 0 = automatic: block_cells, and
                              2*block_cells on a mesh of fewer than 256
                              blocks (latency-bound) (0)                     */
    int32_t load_schedule; /* 0: edge and cell geometry read only where it
                              can change the result (not between cells
                              holding no water) (default); 1: all geometry
                              requested with the state, before the first
                              barrier. Same results; a tuning switch          */
    int32_t monitors;      /* 1: every step also updates the discharge
                              monitors and the flood envelope (see
                              swe_get_discharge, swe_get_envelope); 0: off
                              (0). Turning it on resets them                 */
    int32_t store_all;     /* 1: every cell stores U^{n+1} every step;
                              0: a cell left unchanged on the quiet dry path
                              (h <= h_dry, no flux) in a block that was quiet
                              for the two previous steps skips its store,
                              since the output buffer already holds the same
                              values (0). Same results; a tuning switch      */
    int32_t graph_steps;   /* 0: one kernel launch per step (default);
                              K > 0, a multiple of 6 (at most 4096): runs of
                              K steps are captured once in a HIP graph and
                              replayed (swe_advance; the ensemble's
                              swe_ens_advance likewise). Same results, bit
                              for bit; fewer launch overheads on small
                              meshes. A changed parameter, end time, stream
                              or step phase triggers a new capture          */
} swe_params;

typedef struct {
    int64_t n_nodes, n_cells, n_edges, n_boundary_edges;
    int64_t n_blocks;          /* mesh blocks of block_cells cells           */
    int64_t n_block_edges;     /* edge records over all blocks (edges on a
                                  block border appear in both blocks)        */
    int32_t block_cells, max_block_edges;
    double min_inradius;       /* smallest inscribed radius [m]              */
    double total_area;         /* sum of cell areas [m^2]                    */
} swe_mesh_stats;

/* Version of this interface (SWE_ABI_VERSION). */
int swe_abi_version(void);

/* Fills *p with the defaults listed in swe_params. */
swe_status swe_default_params(swe_params *p);

/* Creates a context bound to HIP device `device` (an ordinal). No device
 * call is made here. *out is owned by the caller and released with
 * swe_destroy. */
swe_status swe_create(swe_ctx **out, int device);

/* Releases the context and every device allocation it made (a workspace
 * bound with swe_bind_workspace stays the caller's). NULL is a no-op. */
void swe_destroy(swe_ctx *ctx);

/* Message of the last failing call on ctx (or of swe_create when ctx is
 * NULL); valid until the next call on ctx. */
const char *swe_last_error(const swe_ctx *ctx);

/* HIP stream (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream)
 * on which every later kernel and copy is issued; NULL = the null stream.
 * The stream must belong to the context's device and outlive its use. */
swe_status swe_set_stream(swe_ctx *ctx, void *hip_stream);

/* Validates and stores parameters. g, cfl, h_dry, dt_max apply from the
 * next step; block_cells and reorder from the next swe_set_mesh. */
swe_status swe_set_params(swe_ctx *ctx, const swe_params *p);
swe_status swe_get_params(const swe_ctx *ctx, swe_params *p);

/* Mesh (sec. 3.1): n_nodes nodes with coordinates xy[2*k], xy[2*k+1];
 * n_cells triangles tri[3*c..3*c+2] in either orientation (a clockwise
 * triangle is reoriented by exchanging its second and third vertex). The
 * boundary condition of a boundary edge is chosen by a tag: n_bnd segments
 * bnd_nodes[2*s], bnd_nodes[2*s+1] (either order) with tag bnd_tag[s] in
 * [0, SWE_MAX_TAG); boundary edges not listed carry tag 0. n_bnd may be 0
 * (bnd_nodes, bnd_tag then may be NULL).
 * Errors: SWE_EMESH for a node index out of range, a repeated vertex, a
 * zero-area triangle, an edge shared by more than two triangles, two
 * triangles on the same side of an edge, a segment that is not a boundary
 * edge or is listed twice, a tag out of range, a non-finite coordinate, a
 * mesh of 2^29 cells or more (the step addresses its per-cell arrays with
 * 32-bit byte offsets).
 * Resets the bathymetry and Manning field to 0, the state to dry, the clock
 * to t = 0 and drops any bound workspace. */
swe_status swe_set_mesh(swe_ctx *ctx, int64_t n_nodes, const double *xy,
                        int64_t n_cells, const int32_t *tri, int64_t n_bnd,
                        const int32_t *bnd_nodes, const int32_t *bnd_tag);

/* The same mesh with its edges given (sec. 3.1: the finite volumes are the
 * triangles, and the fluxes cross their edges; the mesh is the node
 * coordinates, the triangles, the edge-to-cell connectivity and the tags of
 * the boundary edges). n_edges edges: edge_nodes[2*e], edge_nodes[2*e+1]
 * (either order), edge_cells[2*e], edge_cells[2*e+1] (the one or two
 * triangles on the edge, in either slot; -1 in the other slot on the
 * boundary), edge_tag[e] (the boundary condition tag of a boundary edge, in
 * [0, SWE_MAX_TAG); 0 on interior edges; NULL: every tag 0). Arrays are
 * caller-owned and copied. The list is validated against the triangles:
 * SWE_EMESH for a node or triangle index out of range, an edge that is not
 * a side of a triangle it names, a triangle side on no listed edge or on
 * two, two edges joining the same nodes, two triangles on the same side of
 * an edge, a tag out of range or nonzero on an interior edge, and every
 * defect swe_set_mesh reports for the triangles. The edges are used as
 * given (no edge search); left/right and normals follow the same rule as
 * swe_set_mesh (left: the triangle whose counter-clockwise boundary runs
 * from the lower to the higher node number), so a run is bitwise that of
 * swe_set_mesh with the boundary edges listed as tagged segments. Resets
 * the context as swe_set_mesh does. */
swe_status swe_set_mesh_edges(swe_ctx *ctx, int64_t n_nodes, const double *xy,
                              int64_t n_cells, const int32_t *tri,
                              int64_t n_edges, const int32_t *edge_nodes,
                              const int32_t *edge_cells,
                              const int32_t *edge_tag);

/* Cell groups for the next swe_set_mesh (with reorder = 1): cells are
 * ordered by group value first and along the space-filling curve within a
 * group. n_cells values in user order (copied; n_cells = 0 clears them); the
 * next swe_set_mesh uses and clears them, and fails with SWE_EINVAL if its
 * cell count differs. Grouping the cells that hold water at the start apart
 * from the dry ones makes blocks wet or dry as a whole: a dry block costs
 * little, and one that borders no changing block is skipped (dormant).
 * Results do not depend on the order; only the speed does. */
swe_status swe_set_cell_groups(swe_ctx *ctx, int64_t n_cells,
                               const uint8_t *group);

/* The same for a wet mask (nonzero: the cell holds water; n_cells values in
 * user order): three groups, the wet cells, the dry cells at most `band`
 * edge-steps (0..64) from a wet cell, and the other dry cells. Blocks of
 * the last group border no wet cell, so they fall dormant (the step skips
 * them) until water comes within reach. Replaces any groups set before;
 * used and cleared by the next swe_set_mesh like them. */
swe_status swe_set_wet_cells(swe_ctx *ctx, int64_t n_cells,
                             const uint8_t *wet, int32_t band);

/* Counts and sizes of the current mesh. */
swe_status swe_mesh_info(const swe_ctx *ctx, swe_mesh_stats *out);

/* Blocks the next step will compute, and the cells they hold (the others
 * are dormant: dry and quiet for two steps, as are the cells of other
 * blocks they share an edge with, and skipped). A measurement aid: the work a step does depends on the state.
 * Synchronises the stream. */
swe_status swe_get_activity(swe_ctx *ctx, int64_t *blocks, int64_t *cells);

/* 64-bit digest (FNV-1a) of the internal mesh the step reads: cell order,
 * areas, inscribed radii, block edge records, normals, lengths, boundary
 * slots and tags. Two ways of giving the same mesh (edges
 * discovered or listed) yield the same digest. Host only. */
swe_status swe_mesh_digest(const swe_ctx *ctx, uint64_t *digest);

/* internal_of_user[c] = position of user cell c in the library's internal
 * (locality) order. */
swe_status swe_get_cell_order(const swe_ctx *ctx, int32_t *internal_of_user);

/* Cell areas |Omega_i| and inscribed radii R_i (sec. 3.1), user order. */
swe_status swe_get_geometry(const swe_ctx *ctx, double *area,
                            double *inradius);

/* Boundary condition of all boundary edges carrying `tag` (sec. 3.1). Every
 * tag starts as SWE_BC_WALL. */
swe_status swe_set_bc(swe_ctx *ctx, int32_t tag, swe_bc_kind kind,
                      double value);

/* Bed elevation z (eq. 4, the b of the paper) per cell [m], finite. */
swe_status swe_set_bathymetry(swe_ctx *ctx, const double *z, swe_mem mem);

/* Manning coefficient m per cell (eq. 5) [s m^-1/3], finite and >= 0. */
swe_status swe_set_manning(swe_ctx *ctx, const double *n, swe_mem mem);

/* State U = (h, hu, hv) per cell; h >= 0, all finite (SWE_ESTATE otherwise;
 * device inputs are checked on the device). Invalidates the pending time
 * step, which is recomputed from this state. */
swe_status swe_set_state(swe_ctx *ctx, const double *h, const double *hu,
                         const double *hv, swe_mem mem);

/* Copies the current state out (user order) and synchronises the stream.
 * Returns SWE_ENUMERIC (the state is still copied out) if a step since the
 * clock was last set produced a non-finite state or an unbounded time step,
 * so that an error deferred by an asynchronous swe_advance surfaces here. */
swe_status swe_get_state(swe_ctx *ctx, double *h, double *hu, double *hv,
                         swe_mem mem);

/* Simulated time and step counter, for resuming a run. */
swe_status swe_set_time(swe_ctx *ctx, double t, int64_t step);
swe_status swe_get_time(swe_ctx *ctx, double *t, double *last_dt,
                        int64_t *step);

/* Advances at most max_steps explicit steps, stopping early when the time
 * reaches t_end (the last step is shortened to land on t_end exactly; pass
 * INFINITY to run exactly max_steps). The time step of each step is
 * CFL * min over wet cells of R_i / (sqrt(g h_i) + |V_i|), bounded by
 * dt_max, computed on the device from the state the step starts from.
 * With t_end = INFINITY the call only enqueues work (no host sync);
 * otherwise the host polls the device clock every check_every steps.
 * *steps_done and *t_now (either may be NULL) are exact after a sync; with
 * t_end = INFINITY they are max_steps and a synchronised time. Returns
 * SWE_ENUMERIC if a step produced a non-finite state or an unbounded time
 * step (all cells dry, dt_max and t_end infinite); with t_end = INFINITY
 * and t_now NULL the call does not wait for the steps, and the error is
 * reported by the next call that synchronises (swe_get_state,
 * swe_get_time, swe_get_diagnostics, or the next swe_advance). */
swe_status swe_advance(swe_ctx *ctx, int64_t max_steps, double t_end,
                       int64_t *steps_done, double *t_now);

/* Frozen time-step schedule (for the adjoint and its finite-difference
 * checks). Advances n steps: with dt non-NULL, step k takes dt[k] (host
 * array, finite, >= 0) instead of the CFL time step, and no end time
 * applies; with dt NULL the CFL time step as in swe_advance (t_end =
 * +INFINITY). dt_out (host, n values, may be NULL) receives the time step of
 * every step taken, so a run recorded with dt = NULL is replayed bit for
 * bit by passing its dt_out back. The state must give bounded time steps.
 * Synchronises the stream. */
swe_status swe_advance_dt(swe_ctx *ctx, int64_t n, const double *dt,
                          double *dt_out);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): swe_advance_dt with the
 * same arguments and results, bit for bit, that allocates nothing. The
 * recorded time steps are staged in a fixed device array of the library
 * (SWE_NOALLOC_MAX_STEPS doubles, 128 KiB, one per GPU, held until the
 * process ends) instead of a buffer the context allocates. Limits and
 * errors, beyond those of swe_advance_dt:
 *  - with dt_out non-NULL, n > SWE_NOALLOC_MAX_STEPS returns SWE_EINVAL
 *    (split the run into several calls);
 *  - the context's device workspace must already exist (bound with
 *    swe_bind_workspace, or allocated by an earlier call such as
 *    swe_advance of 0 steps), else SWE_ENOTREADY.
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (contexts on different streams or threads) race on it. Synchronises the
 * stream, as swe_advance_dt does. */
#define SWE_NOALLOC_MAX_STEPS 16384
swe_status swe_advance_dt_noalloc(swe_ctx *ctx, int64_t n, const double *dt,
                                  double *dt_out);

/* Discrete adjoint of a gauge misfit, for inverse analysis (calibrating
 * friction and bed against observed depths). From the current state, runs
 * `steps` ordinary steps (time steps recorded), evaluates
 *   *loss = sum over k of (h(gauges[k]) - h_target[k])^2
 * at the end, and returns its gradients with respect to the Manning
 * coefficient and the bed elevation of every cell (user order, host arrays
 * of n_cells; either may be NULL), with the time-step schedule of the run
 * held fixed. The reverse sweep restores states from checkpoints taken
 * every K = `checkpoint_every` steps and replays each segment with its
 * recorded time steps; K = 1 keeps every state and replays nothing. With
 * checkpoint_every = 0 the library picks the smallest K whose states fit in
 * half the free device memory, and at most ceil(sqrt(steps)) (the least
 * memory). Any K gives the same bits. The derivative is that of the
 * branches the forward run takes (wet/dry, wave-speed cases, star region,
 * reconstruction maximum, positivity fix). Afterwards the context holds the
 * final state, time and ledger of the forward run; monitors are reset.
 * The forward steps also keep the sum of each cell's edge contributions,
 * so that the reverse of the cell update needs no second edge evaluation.
 * Needs block_cells = 256; allocates its scratch for the call: about
 * (2 K + steps / K + 4) x 24 B per cell for K > 1, (2 steps + 6) x 24 B
 * per cell for K = 1. Synchronises the stream. */
swe_status swe_adjoint_gauges(swe_ctx *ctx, int64_t steps, int32_t n_gauges,
                              const int32_t *gauges, const double *h_target,
                              int32_t checkpoint_every, double *loss,
                              double *grad_manning, double *grad_z);

/* Total water volume sum |Omega_i| h_i [m^3], the volume added by the
 * positivity fix since the mesh was set [m^3], and the number of cells
 * with h > h_dry. Synchronises the stream; returns SWE_ENUMERIC (values
 * still written) after a failed step, as swe_get_state. */
swe_status swe_get_diagnostics(swe_ctx *ctx, double *mass, double *ledger,
                               int64_t *n_wet);

/* Asynchronous copy of the discharge monitors (sec. 5.3.2: the inflow and
 * outflow rates go to the host while the steps go on). Enqueues, on a
 * stream of the library's own ordered after every step enqueued so far,
 * the per-tag sums of rate and volume (summed as swe_get_discharge does:
 * the same bits) and their copy into out (host, 2 * SWE_MAX_TAG doubles:
 * out[2 t] = rate of tag t [m^3/s], out[2 t + 1] = volume [m^3]; pinned
 * host memory makes the copy overlap the steps). Returns at once. Steps
 * enqueued afterwards wait only for the sums (a few microseconds), not
 * for the copy, and do not change the values copied. out must stay valid
 * until swe_discharge_wait reports the copy done. One copy at a time per
 * context: SWE_ENOTREADY while one is pending, or with monitors off. */
swe_status swe_discharge_async(swe_ctx *ctx, double *out);
/* Completion of the pending asynchronous discharge copy: with block != 0
 * waits for it; else *done (may be NULL) = 1 if it has landed (or none is
 * pending), 0 if not yet. */
swe_status swe_discharge_wait(swe_ctx *ctx, int32_t block, int32_t *done);
/* Discharge monitors and flood envelope (swe_params.monitors = 1), the
 * outflow and inflow rates of a river reach and the maximum-depth map from
 * which flood lines are drawn (sec. 5). Both are reset to the current state
 * when monitors are turned on, when the state is set and by
 * swe_reset_monitors().
 *
 * swe_get_discharge: for boundary tag `tag`, *rate = the volume leaving the
 * domain per unit time through the tag's edges during the last step,
 * sum of L_e G_1 over the edges (G_1 = the normal mass flux of the edge's
 * boundary flux, outward positive; an inflow tag gives -Q) [m^3/s], and
 * *volume = sum over steps of dt times that rate since the last reset [m^3].
 * With the positivity ledger they close the water balance:
 *   mass(t) - mass(t_reset) = -(sum of volumes over tags) + ledger change.
 * Either pointer may be NULL. Synchronises the stream.
 *
 * swe_get_envelope: per cell (user order) the highest depth h reached since
 * the reset (the reset state included) and the first simulated time at the
 * end of a step with h > h_dry (the reset time for cells wet at the reset,
 * +INFINITY for cells never wet). Synchronises the stream.
 *
 * Both return SWE_ENOTREADY while monitors are off. */
swe_status swe_reset_monitors(swe_ctx *ctx);
swe_status swe_get_discharge(swe_ctx *ctx, int32_t tag, double *rate,
                             double *volume);
swe_status swe_get_envelope(swe_ctx *ctx, double *h_max, double *t_wet,
                            swe_mem mem);

/* ------------------------------------------------------------------------
 * Batched ensemble. The uncertainty studies behind the flood lines of
 * sec. 6.4.3 run the solver hundreds of times with sampled inflow and
 * friction; each run is a small mesh that leaves most of the GPU idle. An
 * ensemble takes n configured contexts (mesh, bathymetry, Manning, boundary
 * conditions, state and time as they stand; the contexts stay usable and
 * independent) and advances all of them with one launch of the step kernel
 * per step. Each member keeps its own time step, clock and end time, and
 * its results are bitwise those of advancing its context alone.
 *
 * swe_ens_create: members must share g, cfl, h_dry, dt_max, block_cells and
 * the device (SWE_EINVAL), and have a mesh (SWE_ENOTREADY); together they
 * hold fewer than 2^29 cells (each member padded to whole blocks) and 2^30
 * block-edge records (SWE_EINVAL). Copies what it
 * needs; nothing is retained. The member's monitors are not kept.
 * Errors of a failed create: swe_ens_last_error(NULL).
 * swe_ens_advance: `steps` steps of every member; t_end[n_members] (NULL:
 * all +INFINITY) stops each member at its own end time exactly (later
 * steps of that member are empty). Asynchronous: only enqueues work.
 * swe_ens_get_state / swe_ens_get_time: one member, user cell order; they
 * synchronise the stream and return SWE_ENUMERIC if that member produced a
 * non-finite state or an unbounded time step.
 * swe_ens_workspace_bytes / swe_ens_bind_workspace: as for a context,
 * before the first advance.
 * swe_ens_info: cells of all members and mesh blocks.
 * swe_ens_get_activity: as swe_get_activity, over all members: blocks the
 * next step computes and the member cells they hold. Synchronises the
 * stream. */
typedef struct swe_ens swe_ens;

swe_status swe_ens_create(swe_ens **out, swe_ctx *const *members,
                          int32_t n_members);
void swe_ens_destroy(swe_ens *ens);
const char *swe_ens_last_error(const swe_ens *ens);
swe_status swe_ens_set_stream(swe_ens *ens, void *hip_stream);
swe_status swe_ens_workspace_bytes(swe_ens *ens, size_t *bytes);
swe_status swe_ens_bind_workspace(swe_ens *ens, void *dev_ptr, size_t bytes);
swe_status swe_ens_advance(swe_ens *ens, int64_t steps, const double *t_end);
swe_status swe_ens_get_state(swe_ens *ens, int32_t member, double *h,
                             double *hu, double *hv, swe_mem mem);
swe_status swe_ens_get_time(swe_ens *ens, int32_t member, double *t,
                            double *last_dt, int64_t *steps);
swe_status swe_ens_info(const swe_ens *ens, int64_t *n_cells,
                        int64_t *n_blocks);
swe_status swe_ens_get_activity(swe_ens *ens, int64_t *blocks,
                                int64_t *cells);

/* Device memory: by default the library allocates it on first use. A
 * caller that owns device memory (e.g. a torch uint8 tensor) can instead
 * bind a workspace of at least swe_workspace_bytes() bytes, 256-byte
 * aligned, after swe_set_mesh and before the first device use; it must
 * stay alive until the next swe_set_mesh or swe_destroy. */
swe_status swe_workspace_bytes(const swe_ctx *ctx, size_t *bytes);
swe_status swe_bind_workspace(swe_ctx *ctx, void *dev_ptr, size_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* SWE_H */
