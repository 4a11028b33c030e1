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
# Algorithmic bytes the method moves per cell-update (FP64 state in and
# out, per-cell bed / friction / 1/area / inscribed radius, ~1.5 edges of
# geometry and connectivity, per-cell edge slots); derivation in the design doc.
ALG_BYTES_PER_CELL = 140
KERNEL_SRC = [os.path.join(ROOT, "paper_2010_14416_amd", "csrc", f)
              for f in ("swe_kernels.hip", "swe_scheme.hpp", "swe_device.hpp",
                        "swe_mesh.hpp")]
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
    if args.workload == "bumps":
        return W.bumps_canal(), ("bumps-canal-1M: 1000x500 squares, dam break "
                                 "onto a dry bed over 20 Gaussian bumps, "
                                 "Manning 0.03")
    return W.dam_break_canal(), "dam-break-canal-4k: 100x20 squares"


def traffic_per_launch(workload_name, n_cells):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on this kernel source and workload size."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256") != kernel_hash() or \
            t.get("n_cells") != n_cells:
        return None
    return t.get("bytes_per_launch")


def copy_bandwidth(mb, reps=5):
    """Reference streaming kernel of known traffic: an elementwise pass that
    reads `mb` MiB of float64 and writes `mb` MiB (b = -a, torch's neg
    kernel; a plain copy may be routed to a DMA engine instead of a kernel).
    Returns GB/s counting read + write bytes."""
    import torch
    n = mb * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * n * 8 / (ms * 1e-3) / 1e9


def cpu_baseline(case, seconds, threads):
    import oracle
    o = oracle.Oracle(case, threads=threads)
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.run(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 200:
            break
    return dict(value=case.n_cells * steps / el, unit="cell-updates/s",
                cores=threads, kind="oracle",
                sample=f"{steps} oracle steps from the initial state of the "
                       f"same {case.n_cells}-cell workload ({el:.1f} s, "
                       f"setup excluded)")


def _read_counter_csv(path, counter):
    """Per-dispatch values of one counter from a rocprofv3 counter-collection
    CSV: {kernel name: [KiB per dispatch, ...]}."""
    import csv
    out = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name", counter) != counter:
                continue
            out.setdefault(row["Kernel_Name"], []).append(
                float(row["Counter_Value"]))
    return out


def pmc_summary(fetch_csv, write_csv, copy_mb, n_cells, out_path):
    """Per-launch HBM traffic of the step kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by the ratio of
    known to counted bytes of the reference streaming kernel."""
    fetch = _read_counter_csv(fetch_csv, "FETCH_SIZE")
    write = _read_counter_csv(write_csv, "WRITE_SIZE")

    def pick(d, key):
        ks = [k for k in d if key in k]
        if not ks:
            raise SystemExit(f"no dispatch of a kernel matching {key!r}")
        vals = [v for k in ks for v in d[k]]
        return sum(vals) / len(vals), len(vals)

    known = copy_mb * (1 << 20)
    cf, _ = pick(fetch, "neg_kernel")
    cw, _ = pick(write, "neg_kernel")
    sf, sw = known / (cf * 1024), known / (cw * 1024)
    f_kib, nf = pick(fetch, "swe_step_kernel")
    w_kib, nw = pick(write, "swe_step_kernel")
    res = dict(kernel="swe_step_kernel", kernel_sha256=kernel_hash(),
               n_cells=n_cells,
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
                    choices=["river", "bumps", "canal", "ensemble",
                             "adjoint"])
    ap.add_argument("--cells", type=int, default=13_000_000)
    ap.add_argument("--block-cells", type=int, default=None,
                    help="cells per block (default: 256; 64 for the "
                         "ensemble, whose members run alone keep 256)")
    ap.add_argument("--block-threads", type=int, default=0,
                    help="0: automatic (= block cells)")
    ap.add_argument("--workers", type=int,
                    default=min(16, os.cpu_count() or 1))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mb", type=int, default=2048,
                    help="size of the reference copy (0: skip)")
    ap.add_argument("--sweep", default="",
                    help="comma list of CELLSxTHREADS[sSCHEDULE][mMONITORS]"
                         "[aSTORE_ALL] variants to time on the same mesh "
                         "before the main run (stderr), e.g. "
                         "256x256,256x256s1,256x256m1,256x256a1")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV",
                                                        "WRITE_CSV"),
                    help="write the step kernel's traffic summary from two "
                         "rocprofv3 counter CSVs and exit (no GPU needed)")
    ap.add_argument("--pmc-out", default=TRAFFIC_FILE)
    ap.add_argument("--pmc-cells", type=int, default=13_004_176,
                    help="cell count of the profiled workload")
    ap.add_argument("--members", type=int, default=256,
                    help="ensemble members (--workload ensemble)")
    ap.add_argument("--solo-sample", type=int, default=16,
                    help="ensemble members also timed one at a time")
    ap.add_argument("--no-every-block", action="store_true",
                    help="skip the second timing with every block computed "
                         "and stored (store_all = 1)")
    ap.add_argument("--wet-band", type=int, default=None,
                    help="dry cells within this many edge-steps of a wet "
                         "cell form their own group (swe_set_wet_cells); "
                         "default: the library's choice (2 from a million "
                         "cells on, else 0; 2 for ensemble members)")
    ap.add_argument("--no-group-wet", action="store_true",
                    help="order cells along the curve only, without first "
                         "grouping the initially wet cells apart")
    ap.add_argument("--fd-directions", type=int, default=32,
                    help="finite-difference checks of the adjoint")

    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"ensemble": 500, "adjoint": 2000}.get(args.workload,
                                                            1000)

    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.copy_mb,
                    args.pmc_cells, args.pmc_out)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the step has no multi-GPU "
              f"decomposition (asked for --gpus {args.gpus}).",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    from paper_2010_14416_amd import Solver

    if args.workload == "ensemble":
        run_ensemble(args)
        return
    if args.workload == "adjoint":
        run_adjoint(args)
        return
    t0 = time.perf_counter()
    case, desc = make_case(args)
    log(f"workload {case.name}: {case.n_cells} cells "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    for shape in filter(None, args.sweep.split(",")):
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
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(sw.stream)
        sw.advance(args.steps)
        e1.record(sw.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        sw.time()
        log(f"sweep {bc}x{bt} schedule {sched} monitors {mon} store_all "
            f"{sall}: {ms:.4f} ms/step, "
            f"{case.n_cells / (ms * 1e-3):.4e} cell-updates/s, "
            f"{ALG_BYTES_PER_CELL * case.n_cells / (ms * 1e-3) / 1e9:.0f} "
            f"GB/s algorithmic")
        sw.close()
        del sw

    t0 = time.perf_counter()
    s = Solver(case, device=0, block_cells=args.block_cells or 256,
               group_wet=not args.no_group_wet, wet_band=args.wet_band,
               params={"block_threads": args.block_threads})
    info = s.info()
    s.advance(1, want_time=True)          # device set-up + first step
    setup_s = time.perf_counter() - t0
    log(f"set-up {setup_s:.1f} s, {info['n_blocks']} blocks, "
        f"{info['n_block_edges']} block edges")
    s.advance(args.warmup, want_time=True)
    stream = s.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    s.advance(args.steps)                 # enqueue only; no host sync
    ev1.record(stream)
    torch.cuda.synchronize()
    elapsed_ms = ev0.elapsed_time(ev1)
    t_sim, last_dt, step = s.time()       # also raises on a numeric fault
    log(f"{args.steps} steps in {elapsed_ms:.2f} ms; t = {t_sim:.4f} s, "
        f"dt = {last_dt:.4g} s")
    # the same steps with every block computed and stored (store_all = 1:
    # no dormant blocks skipped, no quiet stores skipped); same results
    every_ms = None
    if not args.no_every_block:
        s.close()
        s = Solver(case, device=0, block_cells=args.block_cells or 256,
                   group_wet=not args.no_group_wet, wet_band=args.wet_band,
                   params={"block_threads": args.block_threads,
                           "store_all": 1})
        s.advance(args.warmup + 1, want_time=True)
        torch.cuda.synchronize()
        ev0.record(s.stream)
        s.advance(args.steps)
        ev1.record(s.stream)
        torch.cuda.synchronize()
        every_ms = ev0.elapsed_time(ev1) / args.steps
        s.time()
        log(f"every block computed: {every_ms:.4f} ms per step")

    copy_gbs = None
    if args.copy_mb > 0:
        copy_gbs = copy_bandwidth(args.copy_mb)
        log(f"reference copy of {args.copy_mb} MiB: {copy_gbs:.0f} GB/s")

    n = case.n_cells
    ms_per_step = elapsed_ms / args.steps
    value = n * args.steps / (elapsed_ms * 1e-3)
    alg_bytes = ALG_BYTES_PER_CELL * n
    achieved = alg_bytes / (ms_per_step * 1e-3) / 1e9
    roofline = dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS,
                    unit="GB/s", frac=achieved / PEAK_HBM_GBS,
                    traffic=traffic_per_launch(case.name, n),
                    copy_gbs=copy_gbs)

    base = None
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", 0) or
                      (os.cpu_count() or 1))
        log(f"cpu baseline: oracle on {threads} threads")
        base = cpu_baseline(case, args.cpu_seconds, threads)
        log(f"cpu baseline {base['value']:.3e} cell-updates/s")
        if threads > 1:
            # the same oracle on one core, a shorter sample
            one = cpu_baseline(case, min(10.0, args.cpu_seconds), 1)
            base["single_core_value"] = one["value"]
            base["single_core_sample"] = one["sample"]
            log(f"cpu baseline, one core: {one['value']:.3e} "
                f"cell-updates/s")

    out = dict(
        metric=METRIC, value=value, unit="cell-updates/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=ms_per_step,
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=desc, n_cells=n, n_edges=info["n_edges"],
                    block_cells=info["block_cells"],
                    block_threads=args.block_threads or info["block_cells"],
                    setup_s=round(setup_s, 2),
                    effective_gbs=achieved,
                    every_block_ms_per_step=every_ms),
        roofline=roofline, cpu_baseline=base)
    print(json.dumps(out), flush=True)
    s.close()


def run_ensemble(args):
    """Batched ensemble of river runs (one launch per step for all members,
    each with its own time step) against the same members advanced one at a
    time: the per-member time of a sample of members run alone, scaled to
    all members, over the ensemble's time."""
    import torch
    import workloads as W
    from paper_2010_14416_amd import Ensemble, Solver

    t0 = time.perf_counter()
    cases = W.ensemble_members(n_members=args.members, steps=args.steps,
                               workers=args.workers)
    n = sum(c.n_cells for c in cases)
    log(f"ensemble: {len(cases)} members, {n} cells "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    t1 = time.perf_counter()
    ens = Ensemble(cases, block_cells=args.block_cells or 64,
                   group_wet=not args.no_group_wet,
                   wet_band=2 if args.wet_band is None else args.wet_band,
                   params={"block_threads": args.block_threads})
    ens.advance(args.warmup)
    ens.time(0)
    setup_s = time.perf_counter() - t1
    info = ens.info()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(ens.stream)
    ens.advance(args.steps)
    ev1.record(ens.stream)
    torch.cuda.synchronize()
    ens_ms = ev0.elapsed_time(ev1)
    for k in range(len(cases)):
        ens.time(k)                       # raises on a numeric fault
    log(f"ensemble: {args.steps} steps in {ens_ms:.2f} ms "
        f"({info['n_blocks']} blocks)")
    ens.close()

    k_sample = max(1, min(args.solo_sample, len(cases)))
    pick = np.linspace(0, len(cases) - 1, k_sample).round().astype(int)
    solo_ms, solo_cells = [], 0
    for k in pick:
        s = Solver(cases[k], device=0, block_cells=args.block_cells or 256,
                   group_wet=not args.no_group_wet, wet_band=args.wet_band,
                   params={"block_threads": args.block_threads})
        s.advance(args.warmup, want_time=True)
        torch.cuda.synchronize()
        ev0.record(s.stream)
        s.advance(args.steps)
        ev1.record(s.stream)
        torch.cuda.synchronize()
        solo_ms.append(ev0.elapsed_time(ev1))
        solo_cells += cases[k].n_cells
        s.time()
        s.close()
    # one at a time, every member: the sample's time per cell-step scaled to
    # all cells, and the sample's mean time per member
    per_member_ms = float(np.mean(solo_ms))
    solo_total_ms = per_member_ms * len(cases)
    log(f"one at a time: {k_sample} members, {per_member_ms:.2f} ms each "
        f"for {args.steps} steps")
    value = n * args.steps / (ens_ms * 1e-3)
    ms_per_step = ens_ms / args.steps
    achieved = ALG_BYTES_PER_CELL * n / (ms_per_step * 1e-3) / 1e9
    out = dict(
        metric=METRIC, value=value, unit="cell-updates/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=ms_per_step,
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=f"ensemble-{len(cases)}: river runs of "
                    "U[10k,200k] cells, Manning U[0.02,0.05], inflow "
                    "U[200,800] m^3/s, own time step each",
                    n_cells=n, members=len(cases), n_blocks=info["n_blocks"],
                    setup_s=round(setup_s, 2), effective_gbs=achieved),
        roofline=dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS,
                      unit="GB/s", frac=achieved / PEAK_HBM_GBS,
                      traffic=None, copy_gbs=None),
        ensemble=dict(one_at_a_time_ms=solo_total_ms,
                      one_at_a_time_ms_per_member=per_member_ms,
                      sampled_members=int(k_sample),
                      ensemble_ms=ens_ms,
                      speedup_vs_one_at_a_time=solo_total_ms / ens_ms),
        cpu_baseline=None)
    print(json.dumps(out), flush=True)


def run_adjoint(args):
    """Inverse case on the 1 M-cell bumps canal: gradient of the squared
    depth misfit at 64 seeded gauge cells after `steps` steps against a
    seeded target run (Manning perturbed), w.r.t. per-cell Manning and bed,
    time steps frozen from the forward run. Timed twice: with the interval
    the library picks (every state kept in HBM when it fits, no replay) and
    with checkpoints every ceil(sqrt(steps)) steps (least memory). Reports
    the adjoint's time per step against the forward's, and the relative
    error against central differences of frozen-schedule runs on seeded
    smooth directions."""
    import torch
    import workloads as W
    from paper_2010_14416_amd import Solver, swe as S

    case = W.bumps_canal()
    steps = args.steps
    rng = np.random.default_rng(np.random.SeedSequence(5))
    wet = np.flatnonzero(case.h > 0.05)
    gauges = rng.choice(wet, size=64, replace=False)
    s = Solver(case, device=0)
    dts = S.swe_advance_dt(s.ctx, steps, None, record=True)
    tgt = case.copy()
    tgt.manning = case.manning * (1.0 + 0.2 * rng.uniform(-1, 1,
                                                          case.n_cells))
    t = Solver(tgt, device=0)
    S.swe_advance_dt(t.ctx, steps, dts)
    target = t.state()[0][gauges]
    t.close()

    def forward_loss(manning=None, z=None):
        c = case.copy()
        if manning is not None:
            c.manning = manning
        if z is not None:
            c.z = z
        f = Solver(c, device=0)
        S.swe_advance_dt(f.ctx, steps, dts)
        h = f.state()[0]
        f.close()
        return float(np.sum((h[gauges] - target) ** 2))

    # forward time per step with the frozen schedule (as in the FD runs)
    f = Solver(case, device=0)
    S.swe_advance_dt(f.ctx, 20, dts[:20])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.swe_advance_dt(f.ctx, steps, dts)
    fwd_s = time.perf_counter() - t0
    f.close()
    def adjoint(every):
        a = Solver(case, device=0)
        torch.cuda.synchronize()
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
        f"(states kept), {adj_sqrt_s * 1e3:.1f} ms with checkpoints every "
        f"{k_sqrt}; same bits: {same}")
    if not same:
        raise SystemExit("the checkpoint interval changed the gradients")
    # central differences on smooth directions (wet cells for Manning)
    c = case.xy[case.tri].mean(axis=1)
    x = (c - c.min(axis=0)) / (c.max(axis=0) - c.min(axis=0))
    wet_mask = case.h > 0.1
    # each direction at eps = 1e-6 and 1e-7: a difference stencil that
    # crosses a kink of the scheme (wet/dry switch, wave-speed case) does
    # not measure the derivative, and the two step sizes rarely both do
    errs = {"m": {1e-6: [], 1e-7: []}, "z": {1e-6: [], 1e-7: []}}
    for k in range(args.fd_directions):
        kx, ky = rng.integers(1, 4, 2)
        d = np.sin(2 * np.pi * kx * x[:, 0] + rng.uniform(0, 6)) * np.cos(
            2 * np.pi * ky * x[:, 1] + rng.uniform(0, 6))
        which = "m" if k % 2 == 0 else "z"
        for eps in (1e-6, 1e-7):
            if which == "m":
                dm = d * wet_mask
                fd = (forward_loss(manning=case.manning + eps * dm) -
                      forward_loss(manning=case.manning - eps * dm)) / (
                          2 * eps)
                ad = float(np.dot(gm, dm))
            else:
                fd = (forward_loss(z=case.z + eps * d) -
                      forward_loss(z=case.z - eps * d)) / (2 * eps)
                ad = float(np.dot(gz, d))
            errs[which][eps].append(abs(ad - fd) / max(abs(fd), 1e-3 * loss))
    errs_m, errs_z = errs["m"][1e-6], errs["z"][1e-6]
    best_m = [min(a, b) for a, b in zip(errs["m"][1e-6], errs["m"][1e-7])]
    best_z = [min(a, b) for a, b in zip(errs["z"][1e-6], errs["z"][1e-7])]
    log(f"finite differences (eps 1e-6): Manning max rel error "
        f"{max(errs_m):.2e} (median {np.median(errs_m):.2e}), bed max "
        f"{max(errs_z):.2e} (median {np.median(errs_z):.2e}); better of "
        f"eps 1e-6, 1e-7: Manning max {max(best_m):.2e}, bed max "
        f"{max(best_z):.2e}")
    # cost of one adjoint step: (forward + reverse) minus the forward, per
    # step, against a forward step
    ratio = (adj_s - fwd_s) / fwd_s
    ratio_sqrt = (adj_sqrt_s - fwd_s) / fwd_s
    out = dict(
        metric=METRIC, value=case.n_cells * steps / adj_s,
        unit="cell-updates/s", n_gpus=1, steps=steps, warmup=20,
        ms_per_step=adj_s * 1e3 / steps, higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload="adjoint-bumps-canal-1M: gauge misfit at 64 "
                    "cells vs a perturbed-Manning target run, gradients "
                    "w.r.t. Manning and bed, frozen time steps, states "
                    "kept in HBM", n_cells=case.n_cells),
        roofline=None, cpu_baseline=None,
        adjoint=dict(loss=loss, forward_ms=fwd_s * 1e3,
                     forward_and_reverse_ms=adj_s * 1e3,
                     reverse_step_vs_forward_step=ratio,
                     sqrt_checkpoints_every=k_sqrt,
                     forward_and_reverse_sqrt_checkpoints_ms=adj_sqrt_s * 1e3,
                     reverse_step_vs_forward_step_sqrt_checkpoints=ratio_sqrt,
                     fd_directions=args.fd_directions, fd_eps=1e-6,
                     fd_max_rel_error_manning=max(errs_m),
                     fd_max_rel_error_bed=max(errs_z),
                     fd_median_rel_error_manning=float(np.median(errs_m)),
                     fd_median_rel_error_bed=float(np.median(errs_z)),
                     fd_eps_pair=[1e-6, 1e-7],
                     fd_max_rel_error_manning_better_eps=max(best_m),
                     fd_max_rel_error_bed_better_eps=max(best_z)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
