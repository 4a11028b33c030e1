// Runs of step launches captured in a HIP graph and replayed (the
// graph_steps parameter of include/swe.h): on small meshes a step takes a
// few microseconds of work, and launching it one kernel at a time costs as
// much again; a graph of K launches is submitted at once.
//
// A step's launch arguments differ from the previous step's only in the
// ping-pong buffers (step parity), the clock slot (step index mod 3) and
// the step index itself, whose parity selects the run marks. Everything the
// kernel needs beyond that (time, step index for the error report, time
// step) it reads from the device clock. A graph of K steps, K a multiple of
// 6, therefore replays correctly whenever the run starts at the phase it
// was captured at (step index mod 6, buffer, clock slot) with the same
// remaining arguments; otherwise the steps run one launch at a time until
// the phase matches, or a new graph is captured.
#include <cstring>

#include "swe_device.hpp"

namespace swe {

namespace {

// The arguments that stay the same from step to step.
bool same_fixed_args(const StepArgs &x, const StepArgs &y)
{
#define SAME(f) (x.f == y.f)
    return SAME(blk_edge) && SAME(be_a) && SAME(be_b) && SAME(be_nx) &&
           SAME(be_ny) && SAME(be_len) && SAME(z) && SAME(gm2) &&
           SAME(area) && SAME(inradius) && SAME(bc) && SAME(clock) &&
           SAME(ledger) && SAME(quiet) && SAME(run) && SAME(act) &&
           SAME(mon) && SAME(blk_member) &&
           SAME(member_end) && SAME(t_end_m) &&
           std::memcmp(&x.g, &y.g, sizeof x.g) == 0 &&
           std::memcmp(&x.cfl, &y.cfl, sizeof x.cfl) == 0 &&
           std::memcmp(&x.h_dry, &y.h_dry, sizeof x.h_dry) == 0 &&
           std::memcmp(&x.dt_max, &y.dt_max, sizeof x.dt_max) == 0 &&
           std::memcmp(&x.t_end, &y.t_end, sizeof x.t_end) == 0 &&
           SAME(n_cells) && SAME(n_blocks) && SAME(blk_base) &&
           SAME(store_all) && SAME(fresh_out) && SAME(run_log) &&
           SAME(r_out);
#undef SAME
}

void step_args_at(StepArgs &a, const StepBuffers &b, int buf, int slot,
                  long long index)
{
    a.h0 = b.h[buf];
    a.hu0 = b.hu[buf];
    a.hv0 = b.hv[buf];
    a.h1 = b.h[buf ^ 1];
    a.hu1 = b.hu[buf ^ 1];
    a.hv1 = b.hv[buf ^ 1];
    a.cur = slot;
    a.step_index = index;
}

}  // namespace

void StepGraph::reset()
{
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    steps = 0;
    phase = -1;
    buf = -1;
    slot = -1;
}

StepGraph::~StepGraph()
{
    reset();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
}

hipError_t StepGraph::capture(const StepArgs &a, const StepBuffers &b,
                              int buf0, int slot0, long long index0, int k,
                              const StepLaunch &l)
{
    reset();
    hipError_t e = hipSuccess;
    if (!capture_stream) {
        // a stream of the library's own: the caller's may be the null
        // stream, on which nothing can be captured
        e = hipStreamCreateWithFlags(&capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            capture_stream = nullptr;
            return e;
        }
    }
    e = hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    StepArgs s = a;
    int bf = buf0, sl = slot0;
    hipError_t le = hipSuccess;
    for (int j = 0; j < k && le == hipSuccess; ++j) {
        step_args_at(s, b, bf, sl, index0 + j);
        le = launch_step(s, l.block_cells, l.threads, l.schedule,
                         capture_stream);
        bf ^= 1;
        sl = sl == 2 ? 0 : sl + 1;
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(capture_stream, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le != hipSuccess ? le : e;
    }
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        exec = nullptr;
        return e;
    }
    steps = k;
    phase = int(index0 % 6);
    buf = buf0;
    slot = slot0;
    key = a;
    launch = l;
    return hipSuccess;
}

hipError_t enqueue_steps(StepArgs &a, const StepBuffers &b, int &buf,
                         int &slot, long long &index, int64_t n,
                         const StepLaunch &l, StepGraph *graph, int k,
                         hipStream_t stream)
{
    int64_t done = 0;
    while (done < n) {
        int lead = -1;   // eager steps before the graph can be replayed
        if (graph && k > 0 && n - done >= k) {
            lead = 0;
            const bool usable = graph->exec && graph->steps == k &&
                                graph->launch.block_cells == l.block_cells &&
                                graph->launch.threads == l.threads &&
                                graph->launch.schedule == l.schedule &&
                                same_fixed_args(graph->key, a);
            if (usable) {
                // steps until the phase the graph was captured at
                lead = (graph->phase - int(index % 6) + 6) % 6;
                if ((buf ^ (lead & 1)) != graph->buf ||
                    (slot + lead) % 3 != graph->slot || n - done - lead < k)
                    lead = -2;   // out of reach: capture anew
            }
            if (!usable || lead == -2) {
                hipError_t e = graph->capture(a, b, buf, slot, index, k, l);
                if (e != hipSuccess) return e;
                lead = 0;
            }
        }
        if (lead == 0) {
            hipError_t e = hipGraphLaunch(graph->exec, stream);
            if (e != hipSuccess) return e;
            // k is a multiple of 6: buffer and slot come back to where
            // they were
            index += k;
            done += k;
            continue;
        }
        const int64_t eager = lead > 0 ? lead : n - done;
        for (int64_t j = 0; j < eager; ++j) {
            step_args_at(a, b, buf, slot, index);
            hipError_t e = launch_step(a, l.block_cells, l.threads,
                                       l.schedule, stream);
            if (e != hipSuccess) return e;
            buf ^= 1;
            slot = slot == 2 ? 0 : slot + 1;
            ++index;
            ++done;
        }
    }
    return hipSuccess;
}

}  // namespace swe
