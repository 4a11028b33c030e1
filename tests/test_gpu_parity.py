"""Parity of the HIP path (through the C interface) with the FP64 oracle.

Tolerances: relative L-infinity per field, max|X_gpu - X_ora| / max|X_ora|,
at most 1e-12 after one step and 1e-9 after a full run. Sizes here span many
blocks with a ragged last block; the full-size workloads are in
test_gpu_fullsize.py.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

ONE_STEP = 1e-12
FULL_RUN = 1e-9


def rel_linf(a, b):
    d = float(np.max(np.abs(a - b))) if a.size else 0.0
    s = float(np.max(np.abs(b))) if b.size else 0.0
    return d / max(s, 1e-300)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def solver(case, **kw):
    from paper_2010_14416_amd import Solver
    return Solver(case, device=0, **kw)


def compare(case, steps, t_end=math.inf, tol=ONE_STEP, **kw):
    say(f"[parity] {case.name} cells={case.n_cells} steps={steps} "
        f"t_end={t_end} {kw}")
    s = solver(case, **kw)
    n_gpu, t_gpu = s.advance(steps, t_end, want_time=True)
    hg, hug, hvg = s.state()
    o = O.Oracle(case)
    n_ora, t_ora = o.run(steps, t_end)
    ho, huo, hvo = o.state()
    errs = [rel_linf(hg, ho), rel_linf(hug, huo), rel_linf(hvg, hvo)]
    say(f"  rel Linf h={errs[0]:.3e} hu={errs[1]:.3e} hv={errs[2]:.3e} "
        f"steps gpu={n_gpu} ora={n_ora} t gpu={t_gpu!r} ora={t_ora!r}")
    assert n_gpu == n_ora
    assert abs(t_gpu - t_ora) <= 1e-12 * max(1.0, abs(t_ora))
    assert max(errs) <= tol, errs
    return s, o


def test_dam_break_one_step():
    compare(W.dam_break_canal(), 1)


def test_dam_break_full_run_to_5s():
    case = W.dam_break_canal()
    s, o = compare(case, 10**6, case.t_end, FULL_RUN)
    t, last_dt, step = s.time()
    assert t == 5.0 and step == o.clock()["step"]


def test_bumps_dry_bed_one_step_and_run():
    case = W.bumps_canal(nx=200, ny=101, steps=300)       # ragged last block
    assert case.n_cells % 256 != 0
    compare(case, 1)
    s, o = compare(case, case.steps, tol=FULL_RUN)
    m_gpu, led_gpu, wet_gpu = s.diagnostics()
    area, _, _ = o.geometry()
    h, _, _ = o.state()
    m_ora = math.fsum(area * h)
    assert abs(m_gpu - m_ora) <= 1e-12 * m_ora
    assert abs(led_gpu - o.clock()["ledger"]) <= 1e-9 * max(
        1e-300, abs(o.clock()["ledger"])) + 1e-15 * m_ora
    assert wet_gpu == int(np.sum(h > case.h_dry))


def test_river_inflow_fixed_stage_wet_dry():
    case = W.river(n_target=120_000, workers=1, steps=200)
    compare(case, 1)
    compare(case, case.steps, tol=FULL_RUN)


def test_lake_at_rest_gpu():
    case = W.lake_at_rest(nx=100, ny=40)
    s = solver(case)
    s.advance(2000)
    h, hu, hv = s.state()
    wet = h > 0
    assert np.max(np.abs(hu)) <= 1e-12 and np.max(np.abs(hv)) <= 1e-12
    assert np.max(np.abs(h[wet] + case.z[wet] - 0.12)) <= 1e-12


@pytest.mark.parametrize("block_cells,reorder,threads,schedule", [
    (64, True, 0, 0), (128, True, 0, 0), (512, True, 0, 0),
    (256, False, 0, 0), (256, True, 512, 0), (64, True, 128, 0),
    (512, True, 1024, 0), (256, True, 0, 1), (128, True, 256, 1),
    (64, True, 0, 1)])
def test_blocking_and_order_do_not_change_bits(block_cells, reorder,
                                               threads, schedule):
    """Per-cell arithmetic is independent of how cells are grouped into
    blocks, ordered and spread over threads: results are bitwise those of
    the default layout."""
    case = W.bumps_canal(nx=90, ny=31, lx=30.0, ly=10.0, x_dam=15.0)
    ref = solver(case)
    ref.advance(60)
    a = ref.state()
    s = solver(case, block_cells=block_cells, reorder=reorder,
               params={"block_threads": threads, "load_schedule": schedule})
    s.advance(60)
    b = s.state()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("name", ["bumps", "river"])
def test_dormant_blocks_and_skipped_stores_change_no_bit(name):
    """Blocks that stay quiet with quiet neighbours are skipped, and quiet
    blocks skip their stores; store_all = 1 turns both off. Same bits over
    runs whose wet/dry fronts cross dry blocks, through a state reset, a
    bathymetry change and a frozen time-step schedule."""
    from paper_2010_14416_amd import swe as S
    case = (W.bumps_canal(nx=120, ny=40, lx=30.0, ly=10.0, x_dam=8.0)
            if name == "bumps" else W.river(n_target=120_000, workers=1))
    say(f"[dormant] {case.name} cells={case.n_cells}")
    a = solver(case, params={"monitors": 1})
    b = solver(case, params={"monitors": 1, "store_all": 1})

    def same():
        for x, y in zip(a.state(), b.state()):
            assert np.array_equal(x, y)
        assert a.time() == b.time()
        for x, y in zip(a.envelope(), b.envelope()):
            assert np.array_equal(x, y)

    for s in (a, b):
        s.advance(150)
    same()
    # a state reset halfway through a run
    h, hu, hv = a.state()
    h2 = h.copy()
    h2[: h.size // 7] += 0.05
    for s in (a, b):
        s.set_state(h2, hu, hv)
        s.advance(60)
    same()
    # a changed bed
    z2 = case.z.copy()
    z2[h2 <= case.h_dry] -= 0.01
    for s in (a, b):
        S.swe_set_bathymetry(s.ctx, z2)
        s.advance(60)
    same()
    # frozen time steps
    dts = S.swe_advance_dt(a.ctx, 40, None, record=True)
    S.swe_advance_dt(b.ctx, 40, dts)
    same()


def test_user_order_without_dormant_blocks_gives_identical_bits():
    """A shuffled mesh kept in user order (reorder = 0): its blocks
    neighbour more blocks than the table holds, so none is ever skipped;
    same bits as the default order, which skips dormant blocks."""
    case = W.river(n_target=30_000, workers=1)        # cells shuffled
    a = solver(case)
    b = solver(case, reorder=False)
    for s in (a, b):
        s.advance(120)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    assert a.time() == b.time()


def test_wet_grouped_order_gives_identical_bits():
    """Cells grouped by their initial wet state (the default) or along the
    curve only: same states, same time, monitors alike."""
    case = W.river(n_target=60_000, workers=1)
    a = solver(case, group_wet=True, params={"monitors": 1})
    b = solver(case, group_wet=False, params={"monitors": 1})
    assert not np.array_equal(S_order(a), S_order(b))
    a.advance(80)
    b.advance(80)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    assert a.time() == b.time()
    for x, y in zip(a.envelope(), b.envelope()):
        assert np.array_equal(x, y)
    for tag in (0, 1, 2):
        # per-slot values are the same bits; a tag sums its slots in block
        # order, which differs
        for x, y in zip(a.discharge(tag), b.discharge(tag)):
            assert abs(x - y) <= 1e-12 * max(abs(x), 1.0)
    ma, la, wa = a.diagnostics()
    mb, lb, wb = b.diagnostics()
    assert wa == wb and abs(ma - mb) <= 1e-12 * ma
    assert abs(la - lb) <= 1e-12 * max(abs(la), 1e-300) + 1e-300


def S_order(s):
    from paper_2010_14416_amd import swe as S
    return S.swe_get_cell_order(s.ctx)


def test_user_cell_permutation_gives_identical_bits():
    case = W.bumps_canal(nx=90, ny=31, lx=30.0, ly=10.0, x_dam=15.0)
    perm = np.random.default_rng(1).permutation(case.n_cells)
    p = case.copy()
    p.tri, p.z, p.manning = case.tri[perm], case.z[perm], case.manning[perm]
    p.h, p.hu, p.hv = case.h[perm], case.hu[perm], case.hv[perm]
    a = solver(case)
    a.advance(40)
    b = solver(p)
    b.advance(40)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x[perm], y)


def test_zero_steps_change_nothing():
    """advance(0) and a zero-length frozen schedule are no-ops, also
    after steps (dormant marks and clock untouched)."""
    from paper_2010_14416_amd import swe as S
    case = W.bumps_canal(nx=60, ny=20, lx=30.0, ly=10.0, x_dam=10.0)
    s = solver(case)
    s.advance(0)
    assert s.time()[0] == 0.0
    for x, y in zip(s.state(), (case.h, case.hu, case.hv)):
        assert np.array_equal(x, y)
    s.advance(30)
    before, t = s.state(), s.time()
    s.advance(0)
    S.swe_advance_dt(s.ctx, 0, np.zeros(0))
    assert s.time() == t
    for x, y in zip(s.state(), before):
        assert np.array_equal(x, y)
    ref = solver(case)
    ref.advance(60)
    s.advance(30)
    for x, y in zip(s.state(), ref.state()):
        assert np.array_equal(x, y)


def test_run_to_run_determinism():
    case = W.river(n_target=50_000, workers=1)
    a = solver(case)
    a.advance(50)
    b = solver(case)
    b.advance(50)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)


def test_device_tensors_workspace_and_stream_kinds():
    import torch
    case = W.bumps_canal(nx=60, ny=20, lx=30.0, ly=10.0, x_dam=15.0)
    dev = torch.device("cuda", 0)
    a = solver(case, workspace="library", stream=None)
    a.advance(30)
    ha = a.state()
    b = solver(case)
    # device-tensor state in, 30 steps, device-tensor state out
    t = [torch.tensor(x, dtype=torch.float64, device=dev)
         for x in (case.h, case.hu, case.hv)]
    b.set_state(*t)
    b.advance(30)
    out = [torch.empty(case.n_cells, dtype=torch.float64, device=dev)
           for _ in range(3)]
    b.state(out)
    for x, y in zip(ha, out):
        assert np.array_equal(x, y.cpu().numpy())


def test_resume_is_bitwise():
    case = W.bumps_canal(nx=60, ny=20, lx=30.0, ly=10.0, x_dam=15.0)
    a = solver(case)
    a.advance(50)
    full = a.state()
    b = solver(case)
    b.advance(20)
    h, hu, hv = b.state()
    t, _, step = b.time()
    c = solver(case)
    c.set_state(h, hu, hv)
    from paper_2010_14416_amd import swe as S
    S.swe_set_time(c.ctx, t, step)
    c.advance(30)
    for x, y in zip(full, c.state()):
        assert np.array_equal(x, y)
    assert c.time()[2] == a.time()[2]


def test_t_end_stops_exactly_and_counts_steps():
    case = W.dam_break_canal()
    from paper_2010_14416_amd import swe as S
    s = solver(case, params={"check_every": 7})
    n, t = s.advance(10**6, 1.2345)
    o = O.Oracle(case)
    n2, t2 = o.run(10**6, 1.2345)
    assert t == 1.2345 and n == n2
    # already at t_end: nothing to do
    n3, t3 = s.advance(10, 1.2345)
    assert n3 == 0 and t3 == 1.2345
    assert S.swe_get_time(s.ctx)[0] == 1.2345


def test_all_dry_without_bound_reports_numeric_error():
    from paper_2010_14416_amd import swe as S
    case = W.dam_break_canal(nx=10, ny=2, lx=10.0, ly=2.0, h_left=0.0,
                             h_right=0.0)
    s = solver(case)
    with pytest.raises(S.SweError) as e:
        s.advance(1, want_time=True)
    assert e.value.status == S.SWE_ENUMERIC
    # with an end time the step is bounded
    s2 = solver(case)
    n, t = s2.advance(5, 0.5)
    assert t == 0.5 and n == 1


def test_tiny_meshes():
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    case = W.Case(name="two-triangles", xy=xy, tri=tri,
                  bnd=np.zeros((0, 2), np.int32),
                  bnd_tag=np.zeros(0, np.int32), bc={},
                  z=np.array([0.0, 0.1]), manning=np.array([0.02, 0.03]),
                  h=np.array([1.0, 0.2]), hu=np.array([0.1, 0.0]),
                  hv=np.array([0.0, -0.05]))
    compare(case, 1)
    compare(case, 40, tol=FULL_RUN)


def test_state_reset_after_quiet_steps_is_bitwise():
    """Dry blocks that stayed quiet for several steps skip their stores; a new
    state written mid-run must not be affected by that: the run continues
    bitwise as a fresh run from the new state."""
    case = W.bumps_canal(nx=90, ny=31, lx=30.0, ly=10.0, x_dam=15.0)
    # the new state differs from the old run on dry cells too (a film below
    # h_dry), so a store wrongly skipped would leave a visible difference
    new = case.copy()
    new.h = np.where(case.h == 0.0, 0.5 * case.h_dry, case.h)
    a = solver(case)
    a.advance(40)
    a.set_state(new.h, new.hu, new.hv)
    from paper_2010_14416_amd import swe as S
    S.swe_set_time(a.ctx, 0.0, 0)
    a.advance(25)
    b = solver(new)
    b.advance(25)
    assert np.any(b.state()[0] == 0.5 * case.h_dry)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    # the same with the state handed over as device tensors
    import torch
    dev = torch.device("cuda", 0)
    c = solver(case)
    c.advance(40)
    c.set_state(*[torch.tensor(x, dtype=torch.float64, device=dev)
                  for x in (new.h, new.hu, new.hv)])
    S.swe_set_time(c.ctx, 0.0, 0)
    c.advance(25)
    for x, y in zip(c.state(), b.state()):
        assert np.array_equal(x, y)


def test_monitors_match_the_oracle_and_leave_the_state_alone():
    case = W.river(n_target=120_000, workers=1, steps=150)
    say(f"[monitors] {case.name} cells={case.n_cells}")
    s = solver(case, params={"monitors": 1})
    s.advance(case.steps)
    ref = solver(case)
    ref.advance(case.steps)
    for x, y in zip(s.state(), ref.state()):
        assert np.array_equal(x, y)
    o = O.Oracle(case)
    o.run(case.steps)
    q_in = case.bc[1][1]
    vols = []
    for tag in (0, 1, 2):
        rg, vg = s.discharge(tag)
        ro, vo = o.discharge(tag)
        say(f"  tag {tag}: rate gpu={rg!r} ora={ro!r} vol gpu={vg!r} "
            f"ora={vo!r}")
        assert abs(rg - ro) <= 1e-9 * q_in
        assert abs(vg - vo) <= 1e-9 * max(abs(vo), q_in * 1e-3)
        vols.append(vg)
    assert abs(s.discharge(1)[0] + q_in) <= 1e-12 * q_in
    hm, tw = s.envelope()
    om, ot = o.envelope()
    assert rel_linf(hm, om) <= FULL_RUN
    assert np.array_equal(np.isfinite(tw), np.isfinite(ot))
    fin = np.isfinite(ot)
    assert np.max(np.abs(tw[fin] - ot[fin]), initial=0.0) <= 1e-12 * max(
        1.0, float(np.max(ot[fin], initial=0.0)))
    assert np.all(hm >= s.state()[0])


def test_discharge_balance_closes_with_the_ledger():
    """Mass change = -(volume out through every tag) + mass added by the
    positivity fix, on the GPU's own monitors, over a run with inflow,
    fixed stage and wet/dry fronts."""
    case = W.river(n_target=120_000, workers=1)
    s = solver(case, params={"monitors": 1})
    m0, led0, _ = s.diagnostics()
    s.advance(200)
    m1, led1, _ = s.diagnostics()
    t = s.time()[0]
    out = sum(s.discharge(tag)[1] for tag in (0, 1, 2))
    q_in = case.bc[1][1]
    say(f"[balance] dm={m1 - m0!r} out={out!r} ledger={led1 - led0!r}")
    assert abs(s.discharge(1)[1] + q_in * t) <= 1e-11 * q_in * t
    assert abs((m1 - m0) - (-out + (led1 - led0))) <= 1e-9 * q_in * t


def test_envelope_is_the_running_maximum_of_the_states():
    """Bitwise: the envelope equals the maximum over the run's own states
    (rising, falling and re-rising cells; reading it mid-run changes
    nothing) and t_wet is the end time of the first step with h > h_dry."""
    case = W.bumps_canal(nx=90, ny=31, lx=30.0, ly=10.0, x_dam=15.0)
    say(f"[envelope] {case.name} cells={case.n_cells}")
    s = solver(case, params={"monitors": 1})
    h = s.state()[0]
    hmax = h.copy()
    twet = np.where(h > case.h_dry, 0.0, np.inf)
    falls = 0
    for k in range(120):
        s.advance(1)
        hn = s.state()[0]
        t = s.time()[0]
        falls += int(np.sum((hn < h) & (h == hmax)))
        twet = np.where(np.isinf(twet) & (hn > case.h_dry), t, twet)
        hmax = np.maximum(hmax, hn)
        h = hn
        if k % 17 == 3 or k == 119:
            hm, tw = s.envelope()
            assert np.array_equal(hm, hmax), k
            assert np.array_equal(tw, twet), k
    assert falls > 0 and np.any(hmax > h)


def test_monitors_closed_canal_reset_and_off():
    from paper_2010_14416_amd import swe as S
    case = W.dam_break_canal()
    s = solver(case)
    with pytest.raises(S.SweError) as e:
        s.discharge(1)
    assert e.value.status == S.SWE_ENOTREADY
    p = S.swe_get_params(s.ctx)
    p.monitors = 1
    S.swe_set_params(s.ctx, p)
    s.advance(30)
    for tag in range(5):
        assert s.discharge(tag) == (0.0, 0.0)
    hm, tw = s.envelope()
    h = s.state()[0]
    assert np.all(hm >= h) and np.all(hm >= case.h - 1e-15)
    # a reset starts over from the current state
    s.reset_monitors()
    hm2, tw2 = s.envelope()
    t = s.time()[0]
    assert np.array_equal(hm2, h)
    assert np.array_equal(tw2, np.where(h > case.h_dry, t, np.inf))


def test_recorded_time_steps_replay_bitwise():
    """A run's time steps, recorded and passed back as a frozen schedule,
    reproduce it bit for bit; the frozen schedule also holds for a changed
    input (the finite-difference checks of the adjoint rely on it)."""
    from paper_2010_14416_amd import swe as S
    case = W.bumps_canal(nx=90, ny=31, lx=30.0, ly=10.0, x_dam=15.0)
    a = solver(case)
    dts = S.swe_advance_dt(a.ctx, 40, None, record=True)
    ref = solver(case)
    ref.advance(40)
    b = solver(case)
    S.swe_advance_dt(b.ctx, 40, dts)
    for x, y, w in zip(a.state(), ref.state(), b.state()):
        assert np.array_equal(x, y) and np.array_equal(x, w)
    assert np.all(dts > 0) and len(set(dts.tolist())) > 1
    p = case.copy()
    p.manning = case.manning * 1.01
    c = solver(p)
    got = S.swe_advance_dt(c.ctx, 40, dts, record=True)
    assert np.array_equal(got, dts)


def test_listed_edges_run_bitwise_like_discovered_edges():
    """A mesh given with its edge list (shuffled edges, swapped slots, tags
    per edge) runs bit for bit like the same mesh given as triangles with
    tagged boundary segments: river with inflow, fixed stage and wet/dry."""
    case = W.river(n_target=120_000, workers=1)
    say(f"[edges] {case.name} cells={case.n_cells}")
    a = solver(case)
    b = solver(case, edges=W.edge_list(case, seed=9))
    for s in (a, b):
        s.advance(80)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    assert a.time() == b.time()
    o = O.Oracle(case)
    o.run(80)
    for x, y in zip(b.state(), o.state()):
        assert rel_linf(x, y) <= FULL_RUN


def test_deferred_numeric_error_surfaces_in_get_state():
    """An asynchronous advance (t_end infinite, no time asked) that hits an
    unbounded time step returns OK; the next synchronising call reports
    it."""
    from paper_2010_14416_amd import swe as S
    case = W.dam_break_canal(nx=10, ny=2, lx=10.0, ly=2.0, h_left=0.0,
                             h_right=0.0)
    s = solver(case)
    s.advance(3)
    with pytest.raises(S.SweError) as e:
        s.state()
    assert e.value.status == S.SWE_ENUMERIC
    s2 = solver(case)
    s2.advance(2)
    with pytest.raises(S.SweError) as e:
        s2.diagnostics()
    assert e.value.status == S.SWE_ENUMERIC


def test_last_time_step_after_landing_on_t_end():
    """The empty steps launched after t_end inside a polling batch leave the
    last time step (the final, shortened one) and the step count as the
    oracle reports them."""
    from paper_2010_14416_amd import swe as S
    case = W.dam_break_canal()
    for every in (1, 5, 64):
        s = solver(case, params={"check_every": every})
        n, t = s.advance(10**6, 2.5)
        o = O.Oracle(case)
        n2, t2 = o.run(10**6, 2.5)
        tg, dtg, kg = S.swe_get_time(s.ctx)
        ck = o.clock()
        assert t == tg == t2 == 2.5 and n == n2 == kg
        assert dtg == ck["last_dt"] and dtg > 0.0, (every, dtg, ck)


def test_device_bed_change_wakes_dormant_blocks():
    """A bed given as device memory re-arms every block as a host bed does:
    lowering the bed under a dry reach held by a fixed stage below its old
    bed starts inflow there, also in blocks that had fallen dormant."""
    import torch
    case = W.bumps_canal(nx=120, ny=40, lx=30.0, ly=10.0, x_dam=6.0)
    case.bc = dict(case.bc)
    case.bc[2] = (W.BC_FIXED_STAGE, -0.5)       # east side, below the bed
    a = solver(case)
    b = solver(case, params={"store_all": 1})
    for s in (a, b):
        s.advance(100)
    x = case.centroids()[:, 0]
    z2 = case.z.copy()
    z2[x > 24.0] = -1.0
    zt = torch.tensor(z2, dtype=torch.float64, device="cuda")
    m0 = a.diagnostics()[0]
    for s in (a, b):
        from paper_2010_14416_amd import swe as S
        S.swe_set_bathymetry(s.ctx, zt)
        s.advance(60)
    for p, q in zip(a.state(), b.state()):
        assert np.array_equal(p, q)
    h = a.state()[0]
    assert a.diagnostics()[0] > m0 and np.any(h[x > 29.0] > 0.1)


def test_asynchronous_discharge_copy():
    """swe_discharge_async: the per-tag rates and volumes of the step it
    follows, the same bits as swe_get_discharge, untouched by the steps
    enqueued after it; into pinned or pageable host memory; one copy at a
    time; refused with monitors off."""
    import torch
    from paper_2010_14416_amd import swe as S
    case = W.river(n_target=60_000, workers=1)
    s = solver(case, params={"monitors": 1})
    s.advance(37)
    ref = {tag: s.discharge(tag) for tag in (0, 1, 2, 3)}
    assert ref[1][0] < 0.0                         # the inflow comes in
    pinned = torch.empty(2 * S.SWE_MAX_TAG, dtype=torch.float64,
                         pin_memory=True)
    S.swe_discharge_async(s.ctx, pinned)
    with pytest.raises(S.SweError) as e:           # one copy at a time
        S.swe_discharge_async(s.ctx, np.empty(2 * S.SWE_MAX_TAG))
    assert e.value.status == S.SWE_ENOTREADY
    s.advance(25)                                  # steps after the copy
    assert S.swe_discharge_wait(s.ctx, block=True)
    out = pinned.numpy()
    for tag, (rate, vol) in ref.items():
        assert out[2 * tag] == rate and out[2 * tag + 1] == vol
    # the later steps went on as usual
    later = {tag: s.discharge(tag) for tag in (1, 2)}
    a = solver(case, params={"monitors": 1})
    a.advance(62)
    assert later == {tag: a.discharge(tag) for tag in (1, 2)}
    for x, y in zip(s.state(), a.state()):
        assert np.array_equal(x, y)
    # pageable memory, polled
    host = np.zeros(2 * S.SWE_MAX_TAG)
    S.swe_discharge_async(s.ctx, host)
    while not S.swe_discharge_wait(s.ctx, block=False):
        pass
    assert host[2] == later[1][0] and host[5] == later[2][1]
    off = solver(case)
    with pytest.raises(S.SweError) as e:
        S.swe_discharge_async(off.ctx, host)
    assert e.value.status == S.SWE_ENOTREADY
