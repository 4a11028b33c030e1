#!/usr/bin/env python3
"""Throughput of the explicit finite-volume shallow-water step on one GPU.

One "step" is one pass of the whole hot path over the mesh: the device-side
time step (CFL min-reduction of the previous step), every edge's HLLC flux
with hydrostatic reconstruction and bed-slope terms, boundary fluxes, the
semi-implicit Manning friction, the conservative update with wet/dry
handling, and the block minimum feeding the next step's time step. The
default workload is the 13 M-cell synthetic river reach (inflow 500 m^3/s,
fixed downstream stage, partly dry floodplain), FP64 throughout.

Prints one JSON line: cell-updates/s over the timed steps (inputs resident
in HBM), the roofline of the step kernel (algorithmic bytes per launch over
the kernel's average duration, measured with HIP events on the stream the
kernel runs on) and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--workload river|bumps|canal]
"""
import argparse
import hashlib
import json
import re
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("cell-updates/s FP64 + HBM GB/s vs peak; ensemble and adjoint "
          "cost vs plain")
PEAK_HBM_GBS = 8000.0           # MI355X HBM3E, published
# Algorithmic bytes the method moves per cell-update in this FP64 / int32
# layout: U^n in 24 + U^{n+1} out 24 + bed, g m^2, 1/area and inscribed
# radius 32 + about 1.5 edges x (normal, length 24 + two cell indices 8) 48
# + per-cell edge references 12.
ALG_BYTES_PER_CELL = 140
KERNEL_SRC = [os.path.join(ROOT, "paper_2010_14416_amd", "csrc", f)
              for f in ("swe_kernels.hip", "swe_scheme.hpp", "swe_device.hpp",
                        "swe_mesh.hpp")] + [
    os.path.join(ROOT, "paper_2010_14416_amd", "build.py")]   # its flags
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    """Hash of the sources the step kernel is compiled from."""
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def make_case(args):
    import workloads as W
    if args.workload == "river":
        return W.river(n_target=args.cells, workers=args.workers), (
            f"river-{args.cells / 1e6:g}M: seeded meandering reach, "
            "jittered-point Delaunay mesh, thalweg + Perlin bed, Manning "
            "U[0.02,0.05], inflow 500 m^3/s, fixed outlet stage, partly dry "
            "floodplain")
    if args.workload == "wetcanal":
        return W.wet_canal(), ("wet-canal-13M: 3600x1806 squares, every cell "
                               "wet and flowing, flat bed, Manning 0.03")
    if args.workload == "bumps":
        return W.bumps_canal(), ("bumps-canal-1M: 1000x500 squares, dam break "
                                 "onto a dry bed over 20 Gaussian bumps, "
                                 "Manning 0.03")
    return W.dam_break_canal(), "dam-break-canal-4k: 100x20 squares"


def counter_record(n_cells):
    """The committed rocprofv3 counter summary of the step kernel, if it was
    taken on this kernel source and a workload of this size (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256") != kernel_hash() or \
            t.get("n_cells") != n_cells:
        return None
    return t


def ev_time(stream, fn):
    """Milliseconds of the work `fn` enqueues on `stream` (HIP events)."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def copy_bandwidth(mb, min_ms=200.0):
    """Reference streaming kernel of known traffic: an elementwise pass that
    reads `mb` MiB of float64 and writes `mb` MiB (b = -a, torch's neg
    kernel; a plain copy may be routed to a DMA engine instead of a kernel),
    repeated back to back for at least `min_ms` (which also brings the GPU
    out of the low-clock state of the host-side set-up before the timed
    steps). Returns GB/s counting read + write bytes."""
    import torch
    n = mb * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    total_ms, reps = 0.0, 0
    while total_ms < min_ms:
        e0.record()
        for _ in range(10):
            torch.neg(a, out=b)
        e1.record()
        torch.cuda.synchronize()
        total_ms += e0.elapsed_time(e1)
        reps += 10
    del a, b
    return 2 * n * 8 * reps / (total_ms * 1e-3) / 1e9


def warmer(case, **kw):
    """Untimed steps of a second context of the same workload, for about
    `ms` right before a timed leg. After seconds of host-side set-up the GPU
    runs this compute-heavy step slower for its first tens of milliseconds
    of such work: the river's first 20 steps took 0.32 ms each from idle,
    0.27 ms after 0.25 s of streaming copies, and 0.25-0.26 ms (as in the
    rest of the run) after 0.2 s of steps of another context. Every timed
    leg, and both sides of every ratio, start from that state."""
    from paper_2010_14416_amd import Solver
    w = Solver(case, device=0, **kw)
    w.advance(1, want_time=True)

    def warm(ms=200.0):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < ms * 1e-3:
            w.advance(50)
            w.time()
    warm.close = w.close
    return warm


def cpu_model():
    """Host CPU model from /proc/cpuinfo (None if unreadable)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_sample(o, n_cells, seconds, min_steps=1, max_steps=200):
    """Oracle steps until `seconds` have passed (at least min_steps);
    returns (cell-updates/s, steps, seconds)."""
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.run(1)
        steps += 1
        el = time.perf_counter() - t0
        if (el >= seconds and steps >= min_steps) or steps >= max_steps:
            break
    return n_cells * steps / el, steps, el


def cpu_baseline(case, seconds, threads, samples=3, single_steps=10):
    """The FP64 oracle on the host: the median of `samples` timed samples
    of about `seconds` each on `threads` threads, and one sample of at
    least `single_steps` steps on one thread. Set-up excluded; the samples
    continue one run from the workload's initial state."""
    import oracle
    o = oracle.Oracle(case, threads=threads)
    vals, desc = [], []
    for _ in range(samples):
        v, n, el = cpu_sample(o, case.n_cells, seconds)
        vals.append(v)
        desc.append(f"{n} steps in {el:.1f} s")
    del o
    out = dict(value=float(np.median(vals)), unit="cell-updates/s",
               cores=threads, kind="oracle",
               sample=f"median of {samples} samples of oracle steps on the "
                      f"same {case.n_cells}-cell workload, continuing one "
                      f"run from its initial state ({'; '.join(desc)}; "
                      f"set-up excluded)",
               samples=vals, cpu_model=cpu_model())
    if threads > 1 and single_steps > 0:
        o1 = oracle.Oracle(case, threads=1)
        v, n, el = cpu_sample(o1, case.n_cells, 0.0, min_steps=single_steps,
                              max_steps=single_steps)
        out["single_core_value"] = v
        out["single_core_sample"] = (f"{n} oracle steps from the initial "
                                     f"state on one thread ({el:.1f} s)")
    return out


def _read_counter_csv(path, counter):
    """Per-dispatch values of one counter from a rocprofv3 counter-collection
    CSV, in dispatch order: {kernel name: [value per dispatch, ...]}."""
    import csv
    rows = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name", counter) != counter:
                continue
            rows.append((int(row.get("Dispatch_Id") or len(rows)),
                         row["Kernel_Name"], float(row["Counter_Value"])))
    out = {}
    for _, name, v in sorted(rows):
        out.setdefault(name, []).append(v)
    return out


def _step_values(d, select=""):
    """Values of the plain step kernel (not the adjoint's fresh-slot
    instantiation) from _read_counter_csv, dispatches lo:hi if `select`."""
    ks = [k for k in d if "swe_step_kernel" in k and not re.search(
        r"swe_step_kernel<\d+, \d+, \w+, \w+, true>", k)]
    if not ks:
        raise SystemExit("no dispatch of the step kernel")
    vals = [v for k in ks for v in d[k]]
    if select:
        lo, hi = (int(x) if x else None for x in select.split(":"))
        vals = vals[lo:hi]
    return vals


def pmc_table(path, select, cells):
    """Every counter of one rocprofv3 --pmc run, averaged over the step
    kernel's dispatches `select` ("lo:hi"), per launch and per computed
    cell-lane (x 64 for the SQ_INSTS_* wave counts)."""
    import csv
    with open(path, newline="") as f:
        names = sorted({r["Counter_Name"] for r in csv.DictReader(f)})
    out = {}
    for c in names:
        vals = _step_values(_read_counter_csv(path, c), select)
        per = sum(vals) / len(vals)
        out[c] = dict(per_launch=per, dispatches=len(vals))
        if cells:
            out[c]["per_cell"] = per * (64 if c.startswith("SQ_INSTS") else
                                        1) / cells
    print(json.dumps(out, indent=1))
    return out


def pmc_summary(fetch_csv, write_csv, copy_mb, n_cells, out_path,
                valu_csv=None, steps="", select=""):
    """Per-launch HBM traffic of the step kernel from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by the
    ratio of known to counted bytes of the reference streaming kernel; with
    valu_csv, the VALU counters of a third run (SQ_INSTS_VALU,
    SQ_INSTS_VALU_TRANS_F64, SQ_BUSY_CU_CYCLES): instructions per launch and
    the share of the kernel's cycles a SIMD spends issuing them (4 cycles
    per wave64 instruction, 16 for the quarter-rate FP64 transcendentals,
    1 024 SIMDs; SQ_BUSY_CU_CYCLES summed over the 256 CUs). `select`
    ("lo:hi") keeps only those dispatches of the step kernel (in dispatch
    order), e.g. the timed steps of the run."""
    fetch = _read_counter_csv(fetch_csv, "FETCH_SIZE")
    write = _read_counter_csv(write_csv, "WRITE_SIZE")

    def pick(d, key):
        if key == "swe_step_kernel":
            vals = _step_values(d, select)
        else:
            vals = [v for k in d if key in k for v in d[k]]
        if not vals:
            raise SystemExit(f"no dispatch of a kernel matching {key!r}")
        return sum(vals) / len(vals), len(vals)

    known = copy_mb * (1 << 20)
    cf, _ = pick(fetch, "neg_kernel")
    cw, _ = pick(write, "neg_kernel")
    sf, sw = known / (cf * 1024), known / (cw * 1024)
    f_kib, nf = pick(fetch, "swe_step_kernel")
    w_kib, nw = pick(write, "swe_step_kernel")
    res = dict(kernel="swe_step_kernel", kernel_sha256=kernel_hash(),
               n_cells=n_cells, steps=steps, dispatches_kept=select,
               fetch_kib_per_launch=f_kib, write_kib_per_launch=w_kib,
               dispatches=dict(fetch=nf, write=nw),
               reference=dict(kernel="torch neg (elementwise, float64)",
                              bytes_read=known, bytes_written=known,
                              fetch_kib=cf, write_kib=cw,
                              fetch_scale=sf, write_scale=sw),
               fetch_bytes_per_launch=f_kib * 1024 * sf,
               write_bytes_per_launch=w_kib * 1024 * sw)
    res["bytes_per_launch"] = (res["fetch_bytes_per_launch"] +
                               res["write_bytes_per_launch"])
    res["bytes_per_cell"] = res["bytes_per_launch"] / n_cells
    if valu_csv:
        v = {c: pick(_read_counter_csv(valu_csv, c), "swe_step_kernel")[0]
             for c in ("SQ_INSTS_VALU", "SQ_INSTS_VALU_TRANS_F64",
                       "SQ_BUSY_CU_CYCLES")}
        issue = (4 * v["SQ_INSTS_VALU"] +
                 12 * v["SQ_INSTS_VALU_TRANS_F64"]) / 1024
        res["valu"] = dict(insts_per_launch=v["SQ_INSTS_VALU"],
                           trans_f64_per_launch=v["SQ_INSTS_VALU_TRANS_F64"],
                           busy_cu_cycles=v["SQ_BUSY_CU_CYCLES"],
                           issue_frac=issue / (v["SQ_BUSY_CU_CYCLES"] / 256))
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (1000; 500 for the ensemble)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="river",
                    choices=["river", "bumps", "canal", "wetcanal",
                             "ensemble", "adjoint"])
    ap.add_argument("--cells", type=int, default=13_000_000)
    ap.add_argument("--run-steps", type=int, default=1000,
                    help="step count of the workload's run: the steps after "
                         "the timed ones are also timed (run average)")
    ap.add_argument("--block-cells", type=int, default=None,
                    help="cells per block (default: 256; the ensemble's "
                         "autotuner picks its own)")
    ap.add_argument("--block-threads", type=int, default=0,
                    help="0: automatic (= block cells)")
    ap.add_argument("--workers", type=int,
                    default=min(16, os.cpu_count() or 1))
    ap.add_argument("--cpu-seconds", type=float, default=4.0,
                    help="length of each of the 3 multi-thread oracle "
                         "samples")
    ap.add_argument("--cpu-single-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mb", type=int, default=2048,
                    help="size of the reference copy (0: skip)")
    ap.add_argument("--legs", default="small,ensemble,adjoint",
                    help="extra legs of the default run, comma list of "
                         "small, ensemble, adjoint (empty: none)")
    ap.add_argument("--sweep", default="",
                    help="comma list of CELLSxTHREADS[sSCHEDULE][mMONITORS]"
                         "[aSTORE_ALL] variants to time on the same mesh "
                         "before the main run (stderr), e.g. "
                         "256x256,256x256s1,256x256m1,256x256a1")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV",
                                                        "WRITE_CSV"),
                    help="write the step kernel's traffic summary from two "
                         "rocprofv3 counter CSVs and exit (no GPU needed)")
    ap.add_argument("--pmc-valu", default=None,
                    help="with --pmc-summary: a third counter CSV with "
                         "SQ_INSTS_VALU, SQ_INSTS_VALU_TRANS_F64, "
                         "SQ_ACTIVE_INST_VALU, SQ_BUSY_CU_CYCLES")
    ap.add_argument("--pmc-steps", default="",
                    help="with --pmc-summary: which steps the counter runs "
                         "covered (recorded in the summary)")
    ap.add_argument("--pmc-dispatches", default="",
                    help="with --pmc-summary: lo:hi, the step-kernel "
                         "dispatches (in order) to average")
    ap.add_argument("--pmc-out", default=TRAFFIC_FILE)
    ap.add_argument("--pmc-table", default=None, metavar="CSV",
                    help="print every counter of one --pmc run for the step "
                         "kernel's dispatches --pmc-dispatches, per launch "
                         "and per cell of --pmc-table-cells")
    ap.add_argument("--pmc-table-cells", type=float, default=None)
    ap.add_argument("--pmc-cells", type=int, default=13_004_176,
                    help="cell count of the profiled workload")
    ap.add_argument("--members", type=int, default=256,
                    help="ensemble members (--workload ensemble)")
    ap.add_argument("--solo-sample", type=int, default=16,
                    help="ensemble members also timed one at a time")
    ap.add_argument("--ens-shape", default=None, metavar="NC,BAND,THREADS",
                    help="ensemble launch shape (block cells, wet band, "
                         "threads per block, 0 = automatic) instead of the "
                         "autotuner's choice")
    ap.add_argument("--no-autotune", action="store_true",
                    help="ensemble: 64-cell blocks, band 2, no tuning")
    ap.add_argument("--no-every-block", action="store_true",
                    help="skip the second timing with every block computed "
                         "and stored (store_all = 1)")
    ap.add_argument("--wet-band", type=int, default=None,
                    help="dry cells within this many edge-steps of a wet "
                         "cell form their own group (swe_set_wet_cells); "
                         "default: the library's choice (2 from a million "
                         "cells on, else 0)")
    ap.add_argument("--no-group-wet", action="store_true",
                    help="order cells along the curve only, without first "
                         "grouping the initially wet cells apart")
    ap.add_argument("--fd-directions", type=int, default=32,
                    help="finite-difference checks of the adjoint")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="steps per captured HIP graph (0: one launch per "
                         "step)")

    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"ensemble": 500, "adjoint": 2000}.get(args.workload,
                                                            1000)

    if args.pmc_table:
        pmc_table(args.pmc_table, args.pmc_dispatches, args.pmc_table_cells)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.copy_mb,
                    args.pmc_cells, args.pmc_out, args.pmc_valu,
                    args.pmc_steps, args.pmc_dispatches)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the step has no multi-GPU "
              f"decomposition (asked for --gpus {args.gpus}).",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import torch  # noqa: F401

    if args.workload == "ensemble":
        out = base_line(args)
        ens = leg_ensemble(args, steps=args.steps, warmup=args.warmup,
                           solo=args.solo_sample, tune=not args.no_autotune)
        out.update(value=ens["value"], ms_per_step=ens["ensemble_ms"] /
                   args.steps, config=ens.pop("config"),
                   roofline=ens.pop("roofline"), ensemble=ens)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "adjoint":
        out = base_line(args)
        adj = leg_adjoint(args, fd_dirs=args.fd_directions)
        out.update(value=adj.pop("value"), steps=adj["steps"],
                   ms_per_step=adj.pop("ms_per_step"),
                   config=adj.pop("config"), adjoint=adj)
        print(json.dumps(out), flush=True)
        return
    out = run_main(args)
    legs = [x for x in args.legs.split(",") if x] if \
        args.workload == "river" else []

    def leg(name, fn):
        # a failing extra leg is reported in the line, not fatal to it
        try:
            out[name] = fn()
        except Exception as e:   # noqa: BLE001
            log(f"{name} leg failed: {e!r}")
            out[name] = {"error": repr(e)}

    def ensemble_leg():
        ens = leg_ensemble(args, steps=100, warmup=10, solo=8, tune=True,
                           tune_sample=24, tune_steps=10)
        ens.pop("config")
        ens.pop("roofline")
        return ens

    def adjoint_leg():
        adj = leg_adjoint(args, fd_dirs=8)
        for k in ("value", "ms_per_step", "config"):
            adj.pop(k)
        return adj

    if "small" in legs:
        leg("small_mesh", lambda: leg_small(args))
    if "ensemble" in legs:
        leg("ensemble", ensemble_leg)
    if "adjoint" in legs:
        leg("adjoint", adjoint_leg)
    print(json.dumps(out), flush=True)


def base_line(args):
    return dict(metric=METRIC, value=None, unit="cell-updates/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=None,
                higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f64", data="synthetic", config=None, roofline=None,
                cpu_baseline=None)


def run_main(args):
    """The step on one mesh: K timed steps after W warm-up steps, the rest
    of the workload's run, every block computed, which blocks ran, the
    roofline and the oracle on the host."""
    from paper_2010_14416_amd import Solver, swe as S
    t0 = time.perf_counter()
    case, desc = make_case(args)
    log(f"workload {case.name}: {case.n_cells} cells "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    for shape in filter(None, args.sweep.split(",")):
        sweep_one(args, case, shape)

    def solver(**params):
        p = {"block_threads": args.block_threads,
             "graph_steps": args.graph_steps}
        p.update(params)
        return Solver(case, device=0, block_cells=args.block_cells or 256,
                      group_wet=not args.no_group_wet,
                      wet_band=args.wet_band, params=p)

    t0 = time.perf_counter()
    s = solver()
    info = s.info()
    s.advance(1, want_time=True)          # device set-up + first step
    setup_s = time.perf_counter() - t0
    log(f"set-up {setup_s:.1f} s, {info['n_blocks']} blocks, "
        f"{info['n_block_edges']} block edges")
    copy_gbs = None
    if args.copy_mb > 0:
        copy_gbs = copy_bandwidth(args.copy_mb)
        log(f"reference copy of {args.copy_mb} MiB: {copy_gbs:.0f} GB/s")
    gpu_warm = warmer(case, block_cells=args.block_cells or 256,
                      group_wet=not args.no_group_wet,
                      wet_band=args.wet_band)
    gpu_warm()
    s.advance(args.warmup, want_time=True)
    elapsed_ms = ev_time(s.stream, lambda: s.advance(args.steps))
    t_sim, last_dt, step = s.time()       # also raises on a numeric fault
    log(f"{args.steps} steps in {elapsed_ms:.2f} ms; t = {t_sim:.4f} s, "
        f"dt = {last_dt:.4g} s")
    # the rest of the workload's run, timed apart: the average over the run
    done = 1 + args.warmup + args.steps
    rest = max(0, args.run_steps - done)
    run_ms = None
    if rest > 0:
        rest_ms = ev_time(s.stream, lambda: s.advance(rest))
        s.time()
        run_ms = (elapsed_ms + rest_ms) / (args.steps + rest)
        log(f"steps {1 + args.warmup}..{args.run_steps}: {run_ms:.4f} ms "
            "per step")
    s.close()
    # the same steps with every block computed and stored (store_all = 1:
    # no dormant blocks skipped, no quiet stores skipped); same results
    every_ms = None
    if not args.no_every_block:
        s = solver(store_all=1)
        s.advance(1, want_time=True)
        gpu_warm()
        s.advance(args.warmup, want_time=True)
        every_ms = ev_time(s.stream, lambda: s.advance(args.steps)) / \
            args.steps
        s.time()
        s.close()
        log(f"every block computed: {every_ms:.4f} ms per step")
    gpu_warm.close()
    # which blocks the timed steps computed (the same steps again, one at a
    # time, each preceded by a count of the blocks marked to run)
    s = solver()
    s.advance(1 + args.warmup, want_time=True)
    run_cells, run_blocks = [], []
    for k in range(max(args.steps, args.run_steps - 1 - args.warmup)):
        b, c = S.swe_get_activity(s.ctx)
        run_blocks.append(b)
        run_cells.append(c)
        s.advance(1)
    s.close()
    n = case.n_cells
    nb = info["n_blocks"]
    cells_timed = float(np.mean(run_cells[:args.steps]))
    blocks_timed = float(np.mean(run_blocks[:args.steps]))
    log(f"blocks computed per timed step: {blocks_timed:.0f} of {nb} "
        f"({blocks_timed / nb:.3f}); over the run "
        f"{np.mean(run_blocks) / nb:.3f}")

    ms_per_step = elapsed_ms / args.steps
    value = n * args.steps / (elapsed_ms * 1e-3)
    achieved = ALG_BYTES_PER_CELL * cells_timed / (ms_per_step * 1e-3) / 1e9
    effective = ALG_BYTES_PER_CELL * n / (ms_per_step * 1e-3) / 1e9
    rec = counter_record(n)
    traffic = rec.get("bytes_per_launch") if rec else None
    roofline = dict(
        bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s",
        frac=achieved / PEAK_HBM_GBS, traffic=traffic,
        alg_bytes_per_launch=ALG_BYTES_PER_CELL * cells_timed,
        cells_computed_per_launch=cells_timed,
        blocks_computed_frac=blocks_timed / nb,
        effective_gbs_all_cells=effective,
        traffic_gbs=(traffic / (ms_per_step * 1e-3) / 1e9
                     if traffic else None),
        traffic_frac=(traffic / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS
                      if traffic else None),
        traffic_steps=rec.get("steps") if rec else None,
        copy_gbs=copy_gbs)
    if rec and rec.get("valu"):
        v = rec["valu"]
        roofline["valu"] = dict(
            bound="valu", insts_per_launch=v.get("insts_per_launch"),
            issue_frac=v.get("issue_frac"), steps=rec.get("steps"))
    if every_ms:
        roofline["every_block"] = dict(
            ms_per_step=every_ms,
            achieved=ALG_BYTES_PER_CELL * n / (every_ms * 1e-3) / 1e9,
            frac=ALG_BYTES_PER_CELL * n / (every_ms * 1e-3) / 1e9 /
            PEAK_HBM_GBS)

    base = None
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", 0) or
                      (os.cpu_count() or 1))
        log(f"cpu baseline: oracle on {threads} threads")
        base = cpu_baseline(case, args.cpu_seconds, threads,
                            single_steps=args.cpu_single_steps)
        log(f"cpu baseline {base['value']:.3e} cell-updates/s (median), "
            f"one core {base.get('single_core_value', 0):.3e}")

    out = base_line(args)
    out.update(
        value=value, ms_per_step=ms_per_step,
        config=dict(workload=desc, n_cells=n, n_edges=info["n_edges"],
                    block_cells=info["block_cells"],
                    block_threads=args.block_threads or (
                        2 * info["block_cells"]
                        if info["n_blocks"] < 256 and info["block_cells"] <= 512
                        else info["block_cells"]),
                    graph_steps=args.graph_steps,
                    setup_s=round(setup_s, 2),
                    timed_steps=f"{1 + args.warmup}..{done - 1}",
                    run_ms_per_step=run_ms,
                    run_steps=args.run_steps,
                    every_block_ms_per_step=every_ms),
        roofline=roofline, cpu_baseline=base)
    return out


def sweep_one(args, case, shape):
    from paper_2010_14416_amd import Solver
    m = re.fullmatch(r"(\d+)x(\d+)(?:s(\d))?(?:m(\d))?(?:a(\d))?",
                     shape.lower())
    if not m:
        raise SystemExit(f"bad sweep entry {shape!r}")
    bc, bt = int(m.group(1)), int(m.group(2))
    sched, mon, sall = (int(m.group(k) or 0) for k in (3, 4, 5))
    sw = Solver(case, device=0, block_cells=bc,
                group_wet=not args.no_group_wet, wet_band=args.wet_band,
                params={"block_threads": bt, "load_schedule": sched,
                        "monitors": mon, "store_all": sall})
    sw.advance(args.warmup + 1, want_time=True)
    # 0.2 s of untimed steps of another context first, as for the main
    # timing (a GPU fresh from host work runs this step slower at first)
    warm = warmer(case, block_cells=bc, group_wet=not args.no_group_wet,
                  wet_band=args.wet_band, params={"block_threads": bt})
    warm()
    warm.close()
    ms = ev_time(sw.stream, lambda: sw.advance(args.steps)) / args.steps
    sw.time()
    log(f"sweep {bc}x{bt} schedule {sched} monitors {mon} store_all "
        f"{sall}: {ms:.4f} ms/step, "
        f"{case.n_cells / (ms * 1e-3):.4e} cell-updates/s, "
        f"{ALG_BYTES_PER_CELL * case.n_cells / (ms * 1e-3) / 1e9:.0f} "
        f"GB/s algorithmic")
    sw.close()


def leg_small(args, steps=1000, graph_steps=96):
    """The 4 000-cell dam-break canal, launch-bound: one launch per step
    against graph replays of `graph_steps` steps (same results)."""
    import workloads as W
    from paper_2010_14416_amd import Solver
    case = W.dam_break_canal()
    res = {}
    for k in (0, graph_steps):
        s = Solver(case, device=0, params={"graph_steps": k})
        s.advance(2 * max(k, 20), want_time=True)   # includes the capture
        t0 = time.perf_counter()                    # 0.2 s of its own steps
        while time.perf_counter() - t0 < 0.2:
            s.advance(960)
            s.time()
        res[k] = ev_time(s.stream, lambda: s.advance(steps)) / steps
        s.time()
        s.close()
    log(f"canal 4 000 cells: {res[0] * 1e3:.2f} us per step one launch "
        f"each, {res[graph_steps] * 1e3:.2f} us with graphs of "
        f"{graph_steps} steps")
    return dict(workload="dam-break canal, 4 000 cells", steps=steps,
                ms_per_step_launches=res[0],
                ms_per_step_graph=res[graph_steps],
                graph_steps=graph_steps,
                speedup=res[0] / res[graph_steps])


def leg_ensemble(args, steps, warmup, solo, tune, tune_sample=32,
                 tune_steps=20):
    """Batched ensemble of 256 river runs (one launch per step for all
    members, each with its own time step), launch shape picked by the
    autotuner on a sample of the members, against the same members run
    one at a time with the plain solver (one launch per step, and graph
    replays)."""
    import workloads as W
    from paper_2010_14416_amd import Ensemble, Solver, swe as S
    t0 = time.perf_counter()
    cases = W.ensemble_members(n_members=args.members, steps=500,
                               workers=args.workers)
    n = sum(c.n_cells for c in cases)
    log(f"ensemble: {len(cases)} members, {n} cells "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    best, table = (64, 2, 0), {}
    if args.ens_shape:
        best = tuple(int(x) for x in args.ens_shape.split(","))
        tune = False
    if tune:
        t0 = time.perf_counter()
        best, table = S.autotune_ensemble(cases, sample=tune_sample,
                                          warmup=5, steps=tune_steps)
        log(f"autotuner ({time.perf_counter() - t0:.1f} s): "
            + ", ".join(f"{bc}/{b}/{t}: {ms:.4f} ms" for (bc, b, t), ms in
                        sorted(table.items())) + f"; best {best}")
    t1 = time.perf_counter()
    ens = Ensemble(cases, block_cells=best[0], wet_band=best[1],
                   group_wet=not args.no_group_wet,
                   params={"block_threads": best[2]})
    ens.advance(warmup)
    ens.time(0)
    setup_s = time.perf_counter() - t1
    info = ens.info()
    # 0.2 s of the ensemble's own steps (untimed) before the timed ones; the
    # members run alone then take the same step range, each after 50 ms of
    # ensemble steps
    pre = warmup
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.2:
        ens.advance(20)
        ens.time(0)
        pre += 20
    ens_ms = ev_time(ens.stream, lambda: ens.advance(steps))
    for k in range(len(cases)):
        ens.time(k)                       # raises on a numeric fault
    log(f"ensemble: {steps} steps in {ens_ms:.2f} ms ({info['n_blocks']} "
        "blocks)")
    # cells the next 10 steps compute (the rest dormant), one step at a time
    act = []
    for _ in range(10):
        act.append(ens.activity()[1])
        ens.advance(1)
    ens.time(0)
    computed = float(np.mean(act))
    log(f"ensemble: cells computed per step {computed:.0f} of {n} "
        f"({computed / n:.3f})")
    k_sample = max(1, min(solo, len(cases)))
    pick = np.linspace(0, len(cases) - 1, k_sample).round().astype(int)
    solo_ms = {0: [], 96: []}
    for k in pick:
        for g in (0, 96):
            s = Solver(cases[k], device=0, params={"graph_steps": g})
            s.advance(pre, want_time=True)
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < 0.05:
                ens.advance(10)
                ens.time(0)
            solo_ms[g].append(ev_time(s.stream, lambda: s.advance(steps)))
            s.time()
            s.close()
    ens.close()
    per = {g: float(np.mean(v)) for g, v in solo_ms.items()}
    log(f"one at a time: {k_sample} members, {per[0]:.2f} ms each for "
        f"{steps} steps ({per[96]:.2f} ms with graphs); steps {pre + 1}.."
        f"{pre + steps} of each run")
    value = n * steps / (ens_ms * 1e-3)
    ms_per_step = ens_ms / steps
    eff = ALG_BYTES_PER_CELL * n / (ms_per_step * 1e-3) / 1e9
    ach = ALG_BYTES_PER_CELL * computed / (ms_per_step * 1e-3) / 1e9
    return dict(
        value=value, members=len(cases), n_cells=n, steps=steps,
        timed_steps=f"{pre + 1}..{pre + steps}",
        ensemble_ms=ens_ms, ms_per_step=ms_per_step,
        cells_computed_frac=computed / n,
        block_cells=best[0], wet_band=best[1], block_threads=best[2],
        autotune={f"cells {bc} band {b} threads {t or bc}": ms
                  for (bc, b, t), ms in table.items()},
        autotune_sample=tune_sample if tune else 0,
        one_at_a_time_ms_per_member=per[0],
        one_at_a_time_ms_per_member_graph=per[96],
        sampled_members=int(k_sample),
        speedup_vs_one_at_a_time=per[0] * len(cases) / ens_ms,
        speedup_vs_one_at_a_time_graph=per[96] * len(cases) / ens_ms,
        config=dict(workload=f"ensemble-{len(cases)}: river runs of "
                    "U[10k,200k] cells, Manning U[0.02,0.05], inflow "
                    "U[200,800] m^3/s, own time step each",
                    n_cells=n, members=len(cases),
                    n_blocks=info["n_blocks"], setup_s=round(setup_s, 2),
                    effective_gbs=eff),
        roofline=dict(bound="hbm", achieved=ach, peak=PEAK_HBM_GBS,
                      unit="GB/s", frac=ach / PEAK_HBM_GBS, traffic=None,
                      cells_computed_per_launch=computed,
                      effective_gbs_all_cells=eff,
                      note="140 B x the cells of the blocks computed per "
                           "step (the 10 steps after the timed ones)"))


def smooth_direction(case, rng):
    """A seeded smooth field sin(2 pi kx x + a) cos(2 pi ky y + b) on the
    canal's cell centroids (x, y scaled to [0, 1])."""
    c = case.xy[case.tri].mean(axis=1)
    x = (c - c.min(axis=0)) / (c.max(axis=0) - c.min(axis=0))
    kx, ky = rng.integers(1, 4, 2)
    return np.sin(2 * np.pi * kx * x[:, 0] + rng.uniform(0, 6)) * np.cos(
        2 * np.pi * ky * x[:, 1] + rng.uniform(0, 6))


def leg_adjoint(args, fd_dirs):
    """Inverse case on the 1 M-cell bumps canal: gradient of the squared
    depth misfit at 64 seeded gauge cells after 2000 steps against a seeded
    target run (Manning perturbed), w.r.t. per-cell Manning and bed, time
    steps frozen from the forward run. Timed with the interval the library
    picks (every state kept when it fits) and with checkpoints every
    ceil(sqrt(steps)) steps; checked against finite differences of
    frozen-schedule runs on seeded smooth directions.

    Finite differences: for each direction d the loss at m + t d for
    t = +-eps, +-eps/2, +-eps/4. On each side the one-sided Richardson
    values at (eps, eps/2) and (eps/2, eps/4) agree where the loss is
    smooth on that side; a branch switch of the scheme inside the stencil
    (a wet/dry threshold, a wave-speed case, the positivity clamp, the
    reconstruction's max) breaks the agreement. Both sides smooth and
    equal: the central Richardson value (4 C(eps/2) - C(eps)) / 3 is the
    reference; one side smooth: that side's value (the adjoint is the
    derivative of the branches taken at m, so it equals the one-sided
    derivative on a side without a switch); neither: the direction is
    reported and not checked."""
    import workloads as W
    from paper_2010_14416_amd import Solver, swe as S
    case = W.bumps_canal()
    steps = 2000
    rng = np.random.default_rng(np.random.SeedSequence(5))
    wet = np.flatnonzero(case.h > 0.05)
    gauges = rng.choice(wet, size=64, replace=False)
    s = Solver(case, device=0)
    dts = S.swe_advance_dt(s.ctx, steps, None, record=True)
    s.close()
    tgt = case.copy()
    tgt.manning = case.manning * (1.0 + 0.2 * rng.uniform(-1, 1,
                                                          case.n_cells))
    t = Solver(tgt, device=0)
    S.swe_advance_dt(t.ctx, steps, dts)
    target = t.state()[0][gauges]
    t.close()

    import torch
    gpu_warm = warmer(case)
    f = Solver(case, device=0)
    S.swe_advance_dt(f.ctx, 20, dts[:20])
    gpu_warm()
    t0 = time.perf_counter()
    S.swe_advance_dt(f.ctx, steps, dts)
    fwd_s = time.perf_counter() - t0

    def adjoint(every):
        a = Solver(case, device=0)
        a.advance(0)
        gpu_warm()
        t0 = time.perf_counter()
        res = S.swe_adjoint_gauges(a.ctx, steps, gauges, target,
                                   checkpoint_every=every)
        el = time.perf_counter() - t0
        a.close()
        return res, el

    k_sqrt = int(math.ceil(math.sqrt(steps)))
    (loss, gm, gz), adj_s = adjoint(0)
    (loss2, gm2, gz2), adj_sqrt_s = adjoint(k_sqrt)
    same = (loss2 == loss and np.array_equal(gm2, gm) and
            np.array_equal(gz2, gz))
    log(f"adjoint: loss {loss:.6e}; forward {fwd_s * 1e3:.1f} ms, "
        f"forward + reverse {adj_s * 1e3:.1f} ms for {steps} steps "
        f"(library's interval), {adj_sqrt_s * 1e3:.1f} ms with checkpoints "
        f"every {k_sqrt}; same bits: {same}")
    gpu_warm.close()
    if not same:
        raise SystemExit("the checkpoint interval changed the gradients")

    # finite differences with one context: new fields, state and clock
    def run_loss(manning, z):
        S.swe_set_manning(f.ctx, manning)
        S.swe_set_bathymetry(f.ctx, z)
        S.swe_set_state(f.ctx, case.h, case.hu, case.hv)
        S.swe_set_time(f.ctx, 0.0, 0)
        S.swe_advance_dt(f.ctx, steps, dts)
        h = f.state()[0]
        acc = 0.0
        for k in range(len(gauges)):        # the library's order of sums
            r = h[gauges[k]] - target[k]
            acc += r * r
        return acc

    f0 = run_loss(case.manning, case.z)
    wet_mask = case.h > 0.1
    eps = 1e-6
    dirs = []
    for k in range(fd_dirs):
        d = smooth_direction(case, rng)
        which = "manning" if k % 2 == 0 else "bed"
        if which == "manning":
            d = d * wet_mask
            ad = float(np.dot(gm, d))
            L = {t: run_loss(case.manning + t * d, case.z)
                 for t in (eps, -eps, eps / 2, -eps / 2, eps / 4, -eps / 4)}
        else:
            ad = float(np.dot(gz, d))
            L = {t: run_loss(case.manning, case.z + t * d)
                 for t in (eps, -eps, eps / 2, -eps / 2, eps / 4, -eps / 4)}
        scale = max(abs(ad), 1e-3 * loss)
        c1 = (L[eps] - L[-eps]) / (2 * eps)
        c2 = (L[eps / 2] - L[-eps / 2]) / eps
        # one-sided Richardson values per side, at (eps, eps/2) and
        # (eps/2, eps/4); a side is smooth when they agree
        sides = {}
        for sgn, name in ((1.0, "plus"), (-1.0, "minus")):
            q = [(L[sgn * h] - f0) / (sgn * h) for h in (eps, eps / 2,
                                                         eps / 4)]
            r1, r2 = 2 * q[1] - q[0], 2 * q[2] - q[1]
            sides[name] = dict(value=r2, smooth=abs(r1 - r2) <= 1e-7 * scale)
        smooth_both = (sides["plus"]["smooth"] and sides["minus"]["smooth"]
                       and abs(sides["plus"]["value"] -
                               sides["minus"]["value"]) <= 1e-7 * scale)
        if smooth_both:
            kind = "smooth"
            ref = [(4 * c2 - c1) / 3]
        else:
            ref = [v["value"] for v in sides.values() if v["smooth"]]
            kind = "branch switch on one side" if ref else \
                "branch switches on both sides"
        dirs.append(dict(
            which=which, kind=kind, adjoint=ad, central=c1,
            one_sided_plus=sides["plus"]["value"],
            one_sided_minus=sides["minus"]["value"],
            rel_error=(min(abs(ad - v) for v in ref) / scale
                       if ref else None),
            rel_error_central=abs(ad - c1) / scale))
    f.close()
    checked = [d for d in dirs if d["rel_error"] is not None]
    unchecked = [i for i, d in enumerate(dirs) if d["rel_error"] is None]
    max_err = max((d["rel_error"] for d in checked), default=None)
    log(f"finite differences, {fd_dirs} directions: "
        f"{sum(d['kind'] == 'smooth' for d in dirs)} smooth, "
        f"{sum(d['kind'] == 'branch switch on one side' for d in dirs)} "
        f"with a branch switch on one side; max relative error over the "
        f"{len(checked)} checked {max_err}; branch switches on both sides "
        f"(not checked): {unchecked}; central differences alone: max "
        f"{max(d['rel_error_central'] for d in dirs):.2e}")
    ratio = (adj_s - fwd_s) / fwd_s
    ratio_sqrt = (adj_sqrt_s - fwd_s) / fwd_s
    return dict(
        value=case.n_cells * steps / adj_s, ms_per_step=adj_s * 1e3 / steps,
        steps=steps, loss=loss, base_loss_fd=f0,
        forward_ms=fwd_s * 1e3, forward_and_reverse_ms=adj_s * 1e3,
        reverse_step_vs_forward_step=ratio,
        sqrt_checkpoints_every=k_sqrt,
        forward_and_reverse_sqrt_checkpoints_ms=adj_sqrt_s * 1e3,
        reverse_step_vs_forward_step_sqrt_checkpoints=ratio_sqrt,
        fd_directions=fd_dirs, fd_eps=[eps, eps / 2, eps / 4],
        fd_checked_directions=len(checked),
        fd_max_rel_error=max_err,
        fd_unchecked_directions=unchecked,
        fd_max_rel_error_central_all=max(d["rel_error_central"]
                                         for d in dirs),
        fd=dirs,
        config=dict(workload="adjoint-bumps-canal-1M: gauge misfit at 64 "
                    "cells vs a perturbed-Manning target run, gradients "
                    "w.r.t. Manning and bed, frozen time steps",
                    n_cells=case.n_cells))


if __name__ == "__main__":
    main()
