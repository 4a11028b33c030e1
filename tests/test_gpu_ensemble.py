"""Batched ensemble on the GPU: every member advances exactly as its own
context would (bitwise), with its own time step, clock and end time."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def members():
    """Ragged mix: closed canal, dry-bed bumps, two river reaches with their
    own inflow and friction, a lake at rest, and a two-cell mesh."""
    r1 = W.river(n_target=30_000, workers=1, inflow_q=300.0)
    r2 = W.river(n_target=12_000, workers=1, inflow_q=750.0)
    r2.manning = np.full(r2.n_cells, 0.045)
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    tiny = W.Case(name="two-triangles", xy=xy, tri=tri,
                  bnd=np.zeros((0, 2), np.int32),
                  bnd_tag=np.zeros(0, np.int32), bc={},
                  z=np.array([0.0, 0.1]), manning=np.array([0.02, 0.03]),
                  h=np.array([1.0, 0.2]), hu=np.array([0.1, 0.0]),
                  hv=np.array([0.0, -0.05]))
    return [W.dam_break_canal(), W.bumps_canal(nx=70, ny=23, lx=30.0,
                                               ly=10.0, x_dam=15.0),
            r1, r2, W.lake_at_rest(nx=40, ny=16), tiny]


def solo(case, steps, t_end=math.inf):
    from paper_2010_14416_amd import Solver
    s = Solver(case, device=0)
    if math.isfinite(t_end):
        s.advance(10**6, t_end)
    else:
        s.advance(steps)
    return s.state(), s.time()


def test_members_match_their_own_runs_bitwise():
    from paper_2010_14416_amd import Ensemble
    cases = members()
    say(f"[ensemble] sizes {[c.n_cells for c in cases]}")
    ens = Ensemble(cases)
    ens.advance(60)
    for k, case in enumerate(cases):
        (h, hu, hv), (t, dt, step) = solo(case, 60)
        eh, ehu, ehv = ens.state(k)
        et, edt, estep = ens.time(k)
        say(f"  member {k} {case.name}: t={et!r} solo {t!r} steps {estep}")
        assert np.array_equal(eh, h) and np.array_equal(ehu, hu)
        assert np.array_equal(ehv, hv)
        assert (et, edt, estep) == (t, dt, step)


@pytest.mark.parametrize("block_cells", [128, 256])
def test_other_block_sizes_match_their_own_runs_bitwise(block_cells):
    """The ragged mix with 128- and 256-cell ensemble blocks (the default is
    64): each member after 120 steps equals, bit for bit, its own run with
    the Solver's defaults."""
    from paper_2010_14416_amd import Ensemble
    cases = members()
    ens = Ensemble(cases, block_cells=block_cells)
    ens.advance(120)
    for k, case in enumerate(cases):
        (h, hu, hv), (t, dt, step) = solo(case, 120)
        eh, ehu, ehv = ens.state(k)
        say(f"  [{block_cells}] member {k} {case.name}: t={t!r}")
        assert np.array_equal(eh, h) and np.array_equal(ehu, hu)
        assert np.array_equal(ehv, hv)
        assert ens.time(k) == (t, dt, step)
    ens.close()


def test_dormant_blocks_change_no_member_bit():
    """The ensemble with dormant-block skipping and store skipping (the
    default) against the ensemble with both off (store_all = 1), over a run
    long enough for dry blocks to fall dormant and fronts to wake them."""
    from paper_2010_14416_amd import Ensemble
    cases = members()
    a = Ensemble(cases)
    b = Ensemble(cases, params={"store_all": 1})
    a.advance(200)
    b.advance(200)
    for k in range(len(cases)):
        for x, y in zip(a.state(k), b.state(k)):
            assert np.array_equal(x, y)
        assert a.time(k) == b.time(k)


def test_activity_is_the_sum_of_the_members_activities():
    """The blocks an ensemble step computes are those its members compute
    alone with the same block size and band: swe_ens_get_activity equals
    the sum of the members' swe_get_activity, as the run goes from every
    block computed to mostly dormant."""
    from paper_2010_14416_amd import Ensemble, Solver, swe as S
    cases = members()
    ens = Ensemble(cases)
    alone = [Solver(c, device=0, block_cells=64, wet_band=2) for c in cases]
    done = 0
    for at in (0, 1, 3, 40, 150):
        if at > done:
            ens.advance(at - done)
            for s in alone:
                s.advance(at - done)
        done = at
        b, c = ens.activity()
        parts = [S.swe_get_activity(s.ctx) for s in alone]
        say(f"  step {at}: ensemble {b} blocks {c} cells; members "
            f"{sum(p[0] for p in parts)} / {sum(p[1] for p in parts)}")
        assert (b, c) == (sum(p[0] for p in parts), sum(p[1] for p in parts))
    assert c < sum(x.n_cells for x in cases)   # some blocks fell dormant
    for s in alone:
        s.close()
    ens.close()


def test_full_size_ensemble_sampled_members_match_their_own_runs():
    """The benchmarked configuration (256 members, 27.7 M cells, the
    Ensemble's defaults): sampled members after 100 steps equal, bit for
    bit, their own runs with the Solver's defaults."""
    from paper_2010_14416_amd import Ensemble
    cases = W.ensemble_members(steps=100)
    say(f"[ensemble full] {len(cases)} members, "
        f"{sum(c.n_cells for c in cases)} cells")
    ens = Ensemble(cases)
    ens.advance(100)
    for k in (0, 57, 128, 255):
        (h, hu, hv), (t, dt, step) = solo(cases[k], 100)
        eh, ehu, ehv = ens.state(k)
        say(f"  member {k}: {cases[k].n_cells} cells, t={t!r}")
        assert np.array_equal(eh, h) and np.array_equal(ehu, hu)
        assert np.array_equal(ehv, hv)
        assert ens.time(k) == (t, dt, step)
    ens.close()


def test_members_stop_at_their_own_end_times():
    from paper_2010_14416_amd import Ensemble
    cases = members()[:4]
    t_end = np.array([1.5, math.inf, 0.7, 2.0])
    ens = Ensemble(cases)
    ens.advance(400, t_end)
    for k, case in enumerate(cases):
        et, _, estep = ens.time(k)
        if math.isfinite(t_end[k]):
            assert et == t_end[k]
            (h, hu, hv), (t, _, step) = solo(case, 0, t_end[k])
        else:
            (h, hu, hv), (t, _, step) = solo(case, 400)
        assert et == t and estep == step
        for x, y in zip(ens.state(k), (h, hu, hv)):
            assert np.array_equal(x, y)


def test_member_matches_the_oracle():
    from paper_2010_14416_amd import Ensemble
    case = W.river(n_target=20_000, workers=1, inflow_q=650.0)
    ens = Ensemble([W.dam_break_canal(), case])
    ens.advance(50)
    o = O.Oracle(case)
    o.run(50)
    for x, y in zip(ens.state(1), o.state()):
        d = float(np.max(np.abs(x - y)))
        assert d <= 1e-9 * max(float(np.max(np.abs(y))), 1e-300)


def test_a_failing_member_is_reported_alone():
    from paper_2010_14416_amd import Ensemble, swe as S
    dry = W.dam_break_canal(nx=10, ny=2, lx=10.0, ly=2.0, h_left=0.0,
                            h_right=0.0)
    ens = Ensemble([W.dam_break_canal(), dry])
    ens.advance(3)
    with pytest.raises(S.SweError) as e:
        ens.time(1)
    assert e.value.status == S.SWE_ENUMERIC
    assert ens.time(0)[2] == 3

