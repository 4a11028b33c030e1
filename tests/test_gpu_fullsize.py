"""Parity at the full workload sizes, in the launch configuration bench.py
times (block_cells 256, Hilbert order, torch stream and workspace).

* 1 000 000-cell bumps canal: one step and the full 2 000-step run against
  the oracle, every cell.
* 13 M-cell river: one step against the oracle, every cell; the full
  1 000-step run against the oracle's own run, every cell, after every
  100 steps (ten tests in a row, each about half a minute of oracle work
  on 16 host threads), and against the stored record of that run at 4 000
  seeded cells
  (tests/golden/river13M_1000steps.json, written by
  tests/golden/make_river_golden.py, which calls only the oracle), plus
  properties that hold at any size.
"""
import hashlib
import json
import math
import os
import sys
import time

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "river13M_1000steps.json")


def rel_linf(a, b):
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))),
                                              1e-300)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def solver(case):
    from paper_2010_14416_amd import Solver
    return Solver(case, device=0)


# ------------------------------------------------------------ bumps 1M

@pytest.fixture(scope="module")
def bumps():
    t0 = time.time()
    case = W.bumps_canal()
    s = solver(case)
    o = O.Oracle(case)
    say(f"[fullsize] bumps canal {case.n_cells} cells ready in "
        f"{time.time() - t0:.1f} s")
    return case, s, o


@pytest.mark.timeout(300)
def test_bumps_1M_one_step_and_full_run(bumps):
    case, s, o = bumps
    s.advance(1)
    o.run(1)
    g, r = s.state(), o.state()
    e1 = [rel_linf(a, b) for a, b in zip(g, r)]
    say(f"  1 step rel Linf {e1}")
    assert max(e1) <= 1e-12
    t0 = time.time()
    _, t = s.advance(case.steps - 1, want_time=True)
    o.run(case.steps - 1)
    say(f"  oracle {case.steps} steps done in {time.time() - t0:.1f} s")
    g, r = s.state(), o.state()
    e = [rel_linf(a, b) for a, b in zip(g, r)]
    say(f"  {case.steps} steps rel Linf {e}, t gpu={t!r} "
        f"ora={o.clock()['t']!r}")
    assert max(e) <= 1e-9
    assert abs(t - o.clock()["t"]) <= 1e-12 * o.clock()["t"]
    m, led, _ = s.diagnostics()
    area, _, _ = o.geometry()
    m0 = math.fsum(area * case.h)
    assert abs(m - m0 - led) <= 1e-12 * m0
    assert abs(led - o.clock()["ledger"]) <= 1e-12 * m0


# ------------------------------------------------------------ river 13M

@pytest.fixture(scope="module")
def river():
    t0 = time.time()
    case = W.river(workers=min(16, os.cpu_count() or 1))   # threads
    say(f"[fullsize] river {case.n_cells} cells generated in "
        f"{time.time() - t0:.1f} s")
    s = solver(case)
    say(f"  solver ready ({time.time() - t0:.1f} s)")
    o = O.Oracle(case)
    say(f"  oracle ready ({time.time() - t0:.1f} s)")
    return case, s, o


def _restart(case, s, o):
    s.set_state(case.h, case.hu, case.hv)
    from paper_2010_14416_amd import swe as S
    S.swe_set_time(s.ctx, 0.0, 0)
    o.set_state(case.h, case.hu, case.hv)
    o.set_time(0.0, 0)


@pytest.mark.timeout(600)
def test_river_13M_one_step(river):
    case, s, o = river
    _restart(case, s, o)
    s.advance(1)
    o.run(1)
    e = [rel_linf(a, b) for a, b in zip(s.state(), o.state())]
    say(f"  river 1 step rel Linf {e}")
    assert max(e) <= 1e-12


@pytest.mark.timeout(600)
def test_river_13M_full_run(river):
    case, s, o = river
    _restart(case, s, o)
    s.advance(case.steps - 1, want_time=True)
    h, hu, hv = s.state()
    _, _, step = s.time()
    assert step == case.steps - 1
    # properties of any valid state
    assert np.all(np.isfinite(h)) and np.all(h >= 0.0)
    assert np.all(hu[h <= case.h_dry] == 0.0)
    assert np.all(hv[h <= case.h_dry] == 0.0)
    s.advance(1)
    g = s.state()
    t_end, _, _ = s.time()
    # the full run against the oracle's own run at seeded cells
    if not os.path.exists(GOLDEN):
        pytest.skip("golden river run not generated")
    with open(GOLDEN) as f:
        gold = json.load(f)
    for name in ("xy", "tri", "z", "manning", "h"):
        a = np.ascontiguousarray(getattr(case, name))
        assert hashlib.sha256(a.tobytes()).hexdigest() == \
            gold["input_sha256"][name], f"regenerated {name} differs"
    idx = np.asarray(gold["samples"]["index"])
    for k, arr in zip(("h", "hu", "hv"), g):
        err = np.max(np.abs(arr[idx] - np.asarray(gold["samples"][k]))) / \
            max(gold["max_abs"][k], 1e-300)
        say(f"  full run, {idx.size} sampled cells: rel Linf {k} = {err:.3e}")
        assert err <= 1e-9
    assert abs(t_end - gold["t"]) <= 1e-12 * gold["t"]
    m, led, _ = s.diagnostics()
    assert abs(m - gold["mass"]) <= 1e-12 * gold["mass"]


@pytest.fixture(scope="module")
def river_parts():
    return {"done": None}


@pytest.mark.timeout(600)
@pytest.mark.parametrize("part", range(10))
def test_river_13M_full_run_every_cell(river, river_parts, part):
    """The headline configuration as bench.py runs it, every cell against
    the oracle after steps 100, 200, ..., 1000 of the run (one part of 100
    steps per test, in order)."""
    case, s, o = river
    if part == 0:
        _restart(case, s, o)
        river_parts["done"] = 0
    assert river_parts["done"] == 100 * part, "parts run in order"
    t0 = time.time()
    s.advance(100)
    n_ora, t_ora = o.run(100)
    t_gpu, _, steps = s.time()
    say(f"  steps {100 * part + 1}..{100 * (part + 1)}: oracle "
        f"{time.time() - t0:.0f} s")
    assert n_ora == 100 and steps == 100 * (part + 1)
    assert abs(t_gpu - t_ora) <= 1e-12 * t_ora
    for k, a, b in zip(("h", "hu", "hv"), s.state(), o.state()):
        err = rel_linf(a, b)
        say(f"  all {case.n_cells} cells: rel Linf {k} = {err:.3e}")
        assert err <= 1e-9
    river_parts["done"] = 100 * (part + 1)

