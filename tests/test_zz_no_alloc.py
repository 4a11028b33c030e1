"""swe_advance_dt_noalloc (the frozen-schedule advance that allocates
nothing) against swe_advance_dt, through the C interface: the same time
steps and states, bit for bit, on two calls in a row (the second shorter,
so the fixed scratch array holds a longer run's time steps from the call
before), for recorded CFL schedules and replayed ones; and its limits."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case():
    return W.bumps_canal(nx=90, ny=31, lx=30.0, ly=10.0, x_dam=15.0)


def _same(a, b):
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    assert a.time() == b.time()


def test_noalloc_matches_advance_dt_on_two_calls():
    from paper_2010_14416_amd import Solver, swe as S
    case = _case()
    say(f"[noalloc] {case.name} cells={case.n_cells} calls of 300 then 40 "
        "steps")
    a = Solver(case, device=0)
    b = Solver(case, device=0)
    for n in (300, 40):
        da = S.swe_advance_dt(a.ctx, n, None, record=True)
        db = S.swe_advance_dt_noalloc(b.ctx, n, None, record=True)
        say(f"  {n} steps: dt[0] {da[0]!r} dt[-1] {da[-1]!r}")
        assert da.shape == db.shape == (n,)
        assert np.array_equal(da, db)
        assert np.all(da > 0)
        _same(a, b)
    # the recorded run also stays with the oracle (same schedule)
    o = O.Oracle(case)
    o.run(340)
    for x, y in zip(b.state(), o.state()):
        d = float(np.max(np.abs(x - y)))
        assert d <= 1e-9 * max(float(np.max(np.abs(y))), 1e-300)
    a.close()
    b.close()


def test_noalloc_replays_a_frozen_schedule_like_advance_dt():
    from paper_2010_14416_amd import Solver, swe as S
    case = _case()
    rec = Solver(case, device=0)
    dts = S.swe_advance_dt(rec.ctx, 120, None, record=True)
    rec.close()
    a = Solver(case, device=0)
    b = Solver(case, device=0)
    # frozen steps with the schedule recorded back, then a shorter call
    # that records nothing
    got_a = S.swe_advance_dt(a.ctx, 120, dts, record=True)
    got_b = S.swe_advance_dt_noalloc(b.ctx, 120, dts, record=True)
    assert np.array_equal(got_a, dts) and np.array_equal(got_b, dts)
    _same(a, b)
    S.swe_advance_dt(a.ctx, 30, dts[:30])
    S.swe_advance_dt_noalloc(b.ctx, 30, dts[:30])
    _same(a, b)
    a.close()
    b.close()


def test_noalloc_limits():
    from paper_2010_14416_amd import Solver, swe as S
    case = _case()
    # no workspace yet (library-owned, not allocated before the first
    # device call): refused, nothing run
    s = Solver(case, device=0, workspace=None)
    with pytest.raises(S.SweError) as e:
        S.swe_advance_dt_noalloc(s.ctx, 5, None, record=True)
    assert e.value.status == S.SWE_ENOTREADY
    s.advance(0)            # an allocating call sets the workspace up
    d = S.swe_advance_dt_noalloc(s.ctx, 5, None, record=True)
    assert np.all(d > 0)
    # more recorded steps than the scratch array holds: refused
    with pytest.raises(S.SweError) as e:
        S.swe_advance_dt_noalloc(s.ctx, 16385, None, record=True)
    assert e.value.status == S.SWE_EINVAL
    assert "16384" in str(e.value)
    s.close()
