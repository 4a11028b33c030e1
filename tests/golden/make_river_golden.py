"""Writes tests/golden/river13M_1000steps.json: the oracle's state after the
full 1 000-step run of the 13 M-cell river workload, sampled at seeded cells.

Calls only the oracle and the workload generators (no GPU code). Run on a
CPU machine (about 30 min on 8 threads):

    python tests/golden/make_river_golden.py [--threads N]

The file records hashes of the generated input arrays so that a consumer can
check it regenerated the same workload, the global maxima of |h|, |hu|, |hv|
(denominators of the relative L-infinity error), the total volume and
positivity ledger, the final time and step count, and (index, h, hu, hv) at
4 000 seeded cells.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(
    os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                   "river13M_1000steps.json")


def case_hashes(case):
    h = {}
    for name in ("xy", "tri", "bnd", "bnd_tag", "z", "manning", "h", "hu",
                 "hv"):
        a = np.ascontiguousarray(getattr(case, name))
        h[name] = hashlib.sha256(a.tobytes()).hexdigest()
    return h


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--samples", type=int, default=4000)
    args = ap.parse_args()
    t0 = time.time()
    case = workloads.river()
    print(f"generated {case.n_cells} cells in {time.time() - t0:.0f} s",
          flush=True)
    o = oracle.Oracle(case, threads=args.threads)
    area, _, _ = o.geometry()
    m0 = math.fsum(area * case.h)
    done = 0
    while done < case.steps:
        n, t = o.run(min(50, case.steps - done))
        done += n
        print(f"step {done} t={t:.4f} ({time.time() - t0:.0f} s)", flush=True)
    h, hu, hv = o.state()
    clk = o.clock()
    idx = np.sort(np.random.default_rng(31).choice(case.n_cells, args.samples,
                                                   replace=False))
    out = dict(
        workload="river", n_cells=case.n_cells, steps=done, t=clk["t"],
        last_dt=clk["last_dt"], ledger=clk["ledger"], mass0=m0,
        mass=math.fsum(area * h), input_sha256=case_hashes(case),
        max_abs=dict(h=float(np.max(np.abs(h))), hu=float(np.max(np.abs(hu))),
                     hv=float(np.max(np.abs(hv)))),
        n_wet=int(np.sum(h > case.h_dry)),
        samples=dict(index=idx.tolist(), h=[float(x) for x in h[idx]],
                     hu=[float(x) for x in hu[idx]],
                     hv=[float(x) for x in hv[idx]]))
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
