"""Steps replayed from captured HIP graphs (swe_params.graph_steps) give the
same bits as one launch per step: with finite end times and host polls,
across calls whose step phase differs from the captured one, after a state
reset, with monitors, for the ensemble, and for a failing step."""
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def solver(case, **kw):
    from paper_2010_14416_amd import Solver
    return Solver(case, device=0, **kw)


def same(a, b):
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    assert a.time() == b.time()


@pytest.mark.parametrize("k", [6, 24])
def test_dam_break_to_t_end_with_polls(k):
    case = W.dam_break_canal()
    say(f"[graph] {case.name} graph_steps={k} to t=5 s")
    a = solver(case, params={"check_every": 64})
    b = solver(case, params={"check_every": 64, "graph_steps": k})
    na, ta = a.advance(10**6, 5.0)
    nb, tb = b.advance(10**6, 5.0)
    assert (na, ta) == (nb, tb) and tb == 5.0
    same(a, b)


def test_river_calls_out_of_phase_and_state_reset():
    case = W.river(n_target=120_000, workers=1)
    say(f"[graph] {case.name} cells={case.n_cells}")
    a = solver(case)
    b = solver(case, params={"graph_steps": 12})
    for n in (7, 50, 31, 25, 12, 1, 40):
        a.advance(n)
        b.advance(n)
    same(a, b)
    # a new state mid-run: the marks and counters are reset outside the
    # graph, the replays go on
    h, hu, hv = case.h.copy(), case.hu.copy(), case.hv.copy()
    h[: case.n_cells // 3] += 0.05
    for s in (a, b):
        s.set_state(h, hu, hv)
        s.advance(60)
    same(a, b)


def test_monitors_with_graphs():
    from paper_2010_14416_amd import swe as S
    case = W.river(n_target=60_000, workers=1)
    a = solver(case, params={"monitors": 1})
    b = solver(case, params={"monitors": 1, "graph_steps": 6})
    a.advance(45)
    b.advance(45)
    same(a, b)
    for tag in (1, 2):
        assert S.swe_get_discharge(a.ctx, tag) == S.swe_get_discharge(b.ctx,
                                                                     tag)
    for x, y in zip(a.envelope(), b.envelope()):
        assert np.array_equal(x, y)


def test_ensemble_with_graphs():
    from paper_2010_14416_amd import Ensemble
    cases = [W.dam_break_canal(), W.river(n_target=30_000, workers=1),
             W.bumps_canal(nx=70, ny=23, lx=30.0, ly=10.0, x_dam=15.0)]
    a = Ensemble(cases)
    b = Ensemble(cases, params={"graph_steps": 24})
    for n in (30, 55):
        a.advance(n)
        b.advance(n)
    for k in range(len(cases)):
        for x, y in zip(a.state(k), b.state(k)):
            assert np.array_equal(x, y)
        assert a.time(k) == b.time(k)


def test_failing_step_reported_at_its_index():
    from paper_2010_14416_amd import swe as S
    case = W.dam_break_canal(nx=10, ny=2, lx=10.0, ly=2.0, h_left=0.0,
                             h_right=0.0)
    msgs = []
    for k in (0, 6):
        s = solver(case, params={"graph_steps": k})
        s.advance(13)
        with pytest.raises(S.SweError) as e:
            s.time()
        assert e.value.status == S.SWE_ENUMERIC
        msgs.append(str(e.value))
    say(f"  {msgs}")
    assert msgs[0] == msgs[1] and "at step 0" in msgs[0]
