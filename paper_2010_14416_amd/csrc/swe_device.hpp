// Device data layout and kernel launchers of the shallow-water step.
// Shared by the HIP kernels (swe_kernels.hip) and the C interface
// (swe_api.cpp); holds no arithmetic of the method.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace swe {

// Boundary condition of one tag (sec. 3.1 and the fixed-level additions).
struct BcEntry {
    int32_t kind;
    int32_t pad;
    double value;   // Q, depth or stage (see include/swe.h)
    double q;       // inflow discharge per unit length, Q / tag length
};

// Lanes of the time-step minimum: blocks combine their minimum into lane
// (workgroup id mod 8), which follows the round-robin dispatch over the 8
// XCDs; each lane has its own 128-byte line.
constexpr int kClockLanes = 8;

// Device-resident clock. Step n reads slot n % 3 and writes slot (n+1) % 3;
// slot (n+2) % 3 is reset by step n for use by step n+1.
struct Clock {
    double t[3];                   // simulated time at the start of a step
    double last_dt;
    long long steps;               // steps with dt > 0
    unsigned int health;           // bit 0: non-finite state, bit 1: dt = inf
    unsigned int pad;
    long long bad_step;            // first step index that raised health
    double dt_ring[8];             // time step of step index k at k mod 8
    long long pad2;
    // bits of min over wet cells of R_i / s_i, per slot and lane
    unsigned long long minrs[3][kClockLanes][16];
    // index of the step that reads a slot (launches since the mesh was
    // set), so that steps replayed from a captured graph know their own
    long long idx[3];
};

// Monitors: per boundary slot the outward volume rate of the last step and
// the volume since the last reset; per block 4 values {first slot, record
// of the first slot, slots, 0}; per cell the highest depth and the first
// time with h > h_dry (+inf: never).
struct MonPtrs {
    double *mon_rate;
    double *mon_vol;
    const int32_t *blk_bnd;
    double *h_max;
    double *t_wet;
};

struct StepArgs {
    // mesh (internal order); block b holds cells [b NC, min((b+1) NC, n))
    const int32_t *blk_edge;
    const int32_t *be_a;      // left side of each block edge (coded)
    const int32_t *be_b;      // right side (coded)
    const double *be_nx;
    const double *be_ny;
    const double *be_len;
    const double *z;
    const double *gm2;        // g m^2 per cell
    const double *area;
    const double *inradius;
    const BcEntry *bc;        // per boundary slot
    // state: U^n in, U^{n+1} out
    const double *h0;
    const double *hu0;
    const double *hv0;
    double *h1;
    double *hu1;
    double *hv1;
    Clock *clock;
    double *ledger;           // per block: mass added by the positivity fix
    int32_t *quiet;           // per block: consecutive steps (capped at 2) in
                              // which every cell took the quiet dry path
    // dormant blocks: run marks for even and odd step indices
    // (2 x n_blocks), and per block NC / 64 words of bits, one per cell:
    // the cells not on the quiet dry path in the block's last computed
    // step. A block runs at step k if it was not quiet for two steps at
    // step k - 1, or if a cell of another block that shares an edge with
    // one of its cells was not quiet at step k - 1 or k - 2.
    uint32_t *run;
    unsigned long long *act;
    // monitors, null when off (read at their point of use, so that their
    // addresses take no scalar registers through the step)
    const MonPtrs *mon;
    // ensembles (all null for one mesh): per block its member, with the
    // sign bit set on the member's first block; per member the end of its
    // cell range and its end time; `clock` then points to one clock per
    // member
    const int32_t *blk_member;
    const int32_t *member_end;
    const double *t_end_m;
    double g, cfl, h_dry, dt_max, t_end;
    int32_t n_cells;
    int32_t n_blocks;         // blocks of this launch, from block blk_base
    int32_t blk_base;
    int32_t store_all;        // 1: every cell stores every step
    int32_t fresh_out;        // 1: the output holds no earlier state (a
                              // fresh slot): every cell stores, and a
                              // dormant block copies its state over
    uint8_t *run_log;         // null, or per block 1 if it ran this step
                              // and 0 if it was dormant (for the adjoint)
    double *r_out;            // null, or per cell the summed edge
                              // contributions R (3 x n_cells: R_h, R_hu,
                              // R_hv; zero for dormant blocks)
    int32_t cur;              // clock slot of this step
    long long step_index;
};

// Bytes of dynamic LDS the step kernel needs per block.
size_t step_lds_bytes(int block_cells);

// schedule 0: inputs that cannot change the result on dry cells are not
// read; 1: the geometry of every edge and cell is requested up front.
hipError_t launch_step(const StepArgs &a, int block_cells, int threads,
                       int schedule, hipStream_t s);
hipError_t launch_clock_set(Clock *c, double t, long long steps,
                            long long step_index, hipStream_t s);
hipError_t launch_slot_reset(Clock *c, int slot, hipStream_t s);
hipError_t launch_min_rs(const double *h, const double *hu, const double *hv,
                         const double *inradius, int64_t n, double g,
                         double h_dry, Clock *c, int cur, hipStream_t s);
hipError_t launch_gather3(const double *a, const double *b, const double *c,
                          double *A, double *B, double *C, const int32_t *idx,
                          int64_t n, hipStream_t s);
hipError_t launch_gather1(const double *a, double *A, const int32_t *idx,
                          int64_t n, hipStream_t s);
hipError_t launch_check_state(const double *h, const double *hu,
                              const double *hv, int64_t n, unsigned *flag,
                              hipStream_t s);
hipError_t launch_check_field(const double *f, int64_t n, int nonneg,
                              unsigned *flag, hipStream_t s);
hipError_t launch_gm2(const double *m, double *gm2, int64_t n, double g,
                      hipStream_t s);
hipError_t launch_diag(const double *h, const double *area, int64_t n,
                       double h_dry, double *part_mass,
                       unsigned long long *part_wet, int nparts,
                       hipStream_t s);
hipError_t launch_fill_u32(unsigned *p, unsigned v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
// h_max = h; t_wet = t where h > h_dry, else +inf
hipError_t launch_envelope_reset(const double *h, int64_t n, double h_dry,
                                 double t, double *h_max, double *t_wet,
                                 hipStream_t s);

constexpr int kDiagThreads = 256;

// Ping-pong state buffers of a step loop.
struct StepBuffers {
    double *h[2], *hu[2], *hv[2];
};

// Launch configuration of the step kernel.
struct StepLaunch {
    int block_cells, threads, schedule;
};

// A captured run of `steps` step launches (swe_graph.cpp).
struct StepGraph {
    hipGraphExec_t exec = nullptr;
    hipStream_t capture_stream = nullptr;
    int steps = 0;
    int phase = -1;   // step index mod 6 of the first captured step
    int buf = -1;     // buffer the first captured step reads
    int slot = -1;    // clock slot the first captured step reads
    StepArgs key{};   // arguments at capture (per-step fields aside)
    StepLaunch launch{};
    StepGraph() = default;
    StepGraph(const StepGraph &) = delete;
    StepGraph &operator=(const StepGraph &) = delete;
    ~StepGraph();
    void reset();
    hipError_t capture(const StepArgs &a, const StepBuffers &b, int buf0,
                       int slot0, long long index0, int k,
                       const StepLaunch &l);
};

// Enqueues n steps of `a` from buffer `buf`, clock slot `slot` and step
// index `index` (all three advanced), one launch per step, or with graph
// non-null and k > 0 (a multiple of 6) through replays of a graph of k
// steps wherever k steps remain.
hipError_t enqueue_steps(StepArgs &a, const StepBuffers &b, int &buf,
                         int &slot, long long &index, int64_t n,
                         const StepLaunch &l, StepGraph *graph, int k,
                         hipStream_t stream);

}  // namespace swe
