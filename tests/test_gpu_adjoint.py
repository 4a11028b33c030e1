"""Discrete adjoint on the GPU (swe_adjoint_gauges): gradients of the gauge
misfit against the adjoint oracle (PyTorch CPU autograd of the oracle's
step) and against central differences of the GPU's own frozen-schedule
runs."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import adjoint as A

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def solver(case, **kw):
    from paper_2010_14416_amd import Solver
    return Solver(case, device=0, **kw)


def problem(case, steps, n_gauges=64, seed=5):
    """Gauges on wet cells and the depths of a run with a perturbed Manning
    field (both seeded), with the CFL schedule of the unperturbed run."""
    from paper_2010_14416_amd import swe as S
    rng = np.random.default_rng(seed)
    wet = np.flatnonzero(case.h > 0.05)
    gauges = rng.choice(wet, size=min(n_gauges, wet.size), replace=False)
    s = solver(case)
    dts = S.swe_advance_dt(s.ctx, steps, None, record=True)
    tgt = case.copy()
    tgt.manning = case.manning * (1.0 + 0.2 * rng.uniform(-1, 1,
                                                          case.n_cells))
    t = solver(tgt)
    S.swe_advance_dt(t.ctx, steps, dts)
    return gauges, t.state()[0][gauges], dts


def gpu_loss(case, dts, gauges, target, manning=None, z=None):
    from paper_2010_14416_amd import swe as S
    c = case.copy()
    if manning is not None:
        c.manning = manning
    if z is not None:
        c.z = z
    s = solver(c)
    S.swe_advance_dt(s.ctx, len(dts), dts)
    h = s.state()[0]
    return float(np.sum((h[gauges] - target) ** 2))


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("name", ["bumps", "river"])
def test_adjoint_matches_the_oracle(name):
    from paper_2010_14416_amd import swe as S
    case = (W.bumps_canal(nx=40, ny=14, lx=30.0, ly=10.0, x_dam=15.0)
            if name == "bumps" else W.river(n_target=6_000, workers=1))
    steps = 30
    gauges, target, dts = problem(case, steps)
    s = solver(case)
    loss, gm, gz = S.swe_adjoint_gauges(s.ctx, steps, gauges, target,
                                        checkpoint_every=7)
    lo, gmo, gzo = A.gauge_misfit(case, dts, gauges, target)
    say(f"[adjoint] {name}: loss gpu={loss!r} ora={lo!r} "
        f"rel Linf dL/dm={rel(gm, gmo):.2e} dL/dz={rel(gz, gzo):.2e}")
    assert abs(loss - lo) <= 1e-9 * lo
    assert rel(gm, gmo) <= 1e-7
    assert rel(gz, gzo) <= 1e-7
    # the context ends at the forward's final state and time
    ref = solver(case)
    S.swe_advance_dt(ref.ctx, steps, dts)
    for x, y in zip(s.state(), ref.state()):
        assert np.array_equal(x, y)
    assert s.time()[0] == ref.time()[0]


def test_checkpoint_interval_does_not_change_bits():
    from paper_2010_14416_amd import swe as S
    case = W.bumps_canal(nx=40, ny=14, lx=30.0, ly=10.0, x_dam=15.0)
    gauges, target, dts = problem(case, 25)
    out = []
    for k in (0, 1, 2, 4, 25):
        s = solver(case)
        out.append(S.swe_adjoint_gauges(s.ctx, 25, gauges, target,
                                        checkpoint_every=k))
    for loss, gm, gz in out[1:]:
        assert loss == out[0][0]
        assert np.array_equal(gm, out[0][1]) and np.array_equal(gz, out[0][2])


def test_manning_gradient_matches_central_differences():
    """Smooth seeded directions on the wet cells; the GPU's frozen-schedule
    runs give the differences."""
    from paper_2010_14416_amd import swe as S
    case = W.river(n_target=20_000, workers=1)
    steps = 60
    gauges, target, dts = problem(case, steps)
    s = solver(case)
    loss, gm, gz = S.swe_adjoint_gauges(s.ctx, steps, gauges, target)
    rng = np.random.default_rng(11)
    c = case.xy[case.tri].mean(axis=1)
    x = (c - c.min(axis=0)) / (c.max(axis=0) - c.min(axis=0))
    wet = case.h > 0.1
    errs = []
    for _ in range(4):
        kx, ky = rng.integers(1, 4, 2)
        d = np.sin(2 * np.pi * kx * x[:, 0] + rng.uniform(0, 6)) * np.cos(
            2 * np.pi * ky * x[:, 1] + rng.uniform(0, 6)) * wet
        eps = 1e-6
        fd = (gpu_loss(case, dts, gauges, target, manning=case.manning +
                       eps * d) -
              gpu_loss(case, dts, gauges, target, manning=case.manning -
                       eps * d)) / (2 * eps)
        errs.append(abs(float(np.dot(gm, d)) - fd) / max(abs(fd),
                                                         1e-3 * loss))
    say(f"[adjoint fd] relative errors {errs}")
    assert max(errs) <= 1e-6


def test_autograd_function_and_a_descent_step():
    """The torch.autograd wrapper returns the adjoint's gradients, and a
    step against them lowers the misfit (inverse analysis of Manning)."""
    import torch
    from paper_2010_14416_amd import swe as S
    case = W.river(n_target=6_000, workers=1)
    steps = 40
    gauges, target, _ = problem(case, steps)
    s = solver(case)
    state = (case.h, case.hu, case.hv)
    m = torch.tensor(case.manning, dtype=torch.float64, requires_grad=True)
    z = torch.tensor(case.z, dtype=torch.float64, requires_grad=True)
    loss = S.gauge_misfit(s, m, z, state, steps, gauges, target)
    loss.backward()
    d = solver(case)
    l2, gm, gz = S.swe_adjoint_gauges(d.ctx, steps, gauges, target)
    assert loss.item() == l2
    assert np.array_equal(m.grad.numpy(), gm)
    assert np.array_equal(z.grad.numpy(), gz)
    with torch.no_grad():
        m2 = m - 1e-3 * m.grad / m.grad.abs().max() * m.abs().max()
    loss2 = S.gauge_misfit(s, m2.clone().requires_grad_(),
                           z.detach().clone().requires_grad_(), state, steps,
                           gauges, target)
    say(f"[inverse] misfit {loss.item()!r} -> {loss2.item()!r}")
    assert loss2.item() < loss.item()


def test_full_size_canal_gradients_and_checkpoints():
    """The benchmarked case, the 1 M-cell bumps canal (200 steps here):
    gradients with every state kept equal those with checkpoints every 15
    steps bit for bit, and agree with one-sided differences of the GPU's
    own frozen-schedule runs on two smooth directions, on a side of the
    base state where the loss is smooth."""
    from paper_2010_14416_amd import swe as S
    case = W.bumps_canal()
    steps = 200
    gauges, target, dts = problem(case, steps)
    say(f"[adjoint full] {case.n_cells} cells, {steps} steps")
    a = solver(case)
    loss, gm, gz = S.swe_adjoint_gauges(a.ctx, steps, gauges, target)
    # the forward with every state kept (each step into a fresh slot,
    # dormant blocks copying their state over) ends where a plain run does
    ref = solver(case)
    S.swe_advance_dt(ref.ctx, steps, dts)
    for x, y in zip(a.state(), ref.state()):
        assert np.array_equal(x, y)
    ref.close()
    a.close()
    b = solver(case)
    l2, gm2, gz2 = S.swe_adjoint_gauges(b.ctx, steps, gauges, target,
                                        checkpoint_every=15)
    b.close()
    assert l2 == loss and np.array_equal(gm2, gm) and np.array_equal(gz2, gz)
    rng = np.random.default_rng(3)
    c = case.xy[case.tri].mean(axis=1)
    x = (c - c.min(axis=0)) / (c.max(axis=0) - c.min(axis=0))
    wet = case.h > 0.1
    f0 = gpu_loss(case, dts, gauges, target)
    assert abs(f0 - loss) <= 1e-13 * loss   # numpy sums in another order
    for which in ("m", "z"):
        kx, ky = rng.integers(1, 4, 2)
        d = np.sin(2 * np.pi * kx * x[:, 0] + rng.uniform(0, 6)) * np.cos(
            2 * np.pi * ky * x[:, 1] + rng.uniform(0, 6))
        if which == "m":
            dd = d * wet
            ad = float(np.dot(gm, dd))

            def at(t):
                return gpu_loss(case, dts, gauges, target,
                                manning=case.manning + t * dd)
        else:
            ad = float(np.dot(gz, d))

            def at(t):
                return gpu_loss(case, dts, gauges, target, z=case.z + t * d)
        # one-sided Richardson values per side (steps eps, eps/2, eps/4): a
        # side is smooth when its two values agree; the adjoint is the
        # derivative of the branches taken at the base state, so it equals
        # the value of a smooth side
        scale = max(abs(ad), 1e-3 * loss)
        est = []
        for sgn in (1.0, -1.0):
            q = [(at(sgn * h) - f0) / (sgn * h) for h in (1e-6, 5e-7,
                                                          2.5e-7)]
            r1, r2 = 2 * q[1] - q[0], 2 * q[2] - q[1]
            est.append((r2, abs(r1 - r2) <= 1e-7 * scale))
        say(f"  {which}: adjoint {ad!r}, one-sided {est}")
        smooth = [v for v, ok in est if ok]
        assert smooth, "a branch switch within 1e-6 on both sides"
        assert min(abs(ad - v) for v in smooth) <= 1e-6 * scale


@pytest.mark.timeout(600)
def test_configured_case_sqrt_checkpoints_and_32_directions():
    """Config 5 as specified: the 1 M-cell canal over 2 000 steps with
    checkpoints every ceil(sqrt(2000)) = 45 steps (the same bits as every
    state kept), and 32 seeded smooth directions (16 Manning on wet cells,
    16 bed) checked against one-sided differences of frozen-schedule runs
    at eps, eps/2, eps/4 (eps = 1e-6) on a side of the base state where the
    loss is smooth; a direction with a branch switch within the stencil on
    both sides is not checked (at most 8 of 32)."""
    from paper_2010_14416_amd import swe as S
    case = W.bumps_canal()
    steps = 2000
    gauges, target, dts = problem(case, steps)
    say(f"[adjoint config 5] {case.n_cells} cells, {steps} steps")
    a = solver(case)
    loss, gm, gz = S.swe_adjoint_gauges(a.ctx, steps, gauges, target,
                                        checkpoint_every=45)
    a.close()
    b = solver(case)
    l1, gm1, gz1 = S.swe_adjoint_gauges(b.ctx, steps, gauges, target,
                                        checkpoint_every=1)
    b.close()
    assert l1 == loss and np.array_equal(gm1, gm) and np.array_equal(gz1, gz)
    f = solver(case)

    def run_loss(manning, z):
        S.swe_set_manning(f.ctx, manning)
        S.swe_set_bathymetry(f.ctx, z)
        S.swe_set_state(f.ctx, case.h, case.hu, case.hv)
        S.swe_set_time(f.ctx, 0.0, 0)
        S.swe_advance_dt(f.ctx, steps, dts)
        h = f.state()[0]
        return float(np.sum((h[gauges] - target) ** 2))

    f0 = run_loss(case.manning, case.z)
    assert abs(f0 - loss) <= 1e-13 * loss
    rng = np.random.default_rng(5)
    c = case.xy[case.tri].mean(axis=1)
    x = (c - c.min(axis=0)) / (c.max(axis=0) - c.min(axis=0))
    wet = case.h > 0.1
    eps = 1e-6
    checked, worst = 0, 0.0
    for k in range(32):
        kx, ky = rng.integers(1, 4, 2)
        d = np.sin(2 * np.pi * kx * x[:, 0] + rng.uniform(0, 6)) * np.cos(
            2 * np.pi * ky * x[:, 1] + rng.uniform(0, 6))
        if k % 2 == 0:
            d = d * wet
            ad = float(np.dot(gm, d))

            def at(t):
                return run_loss(case.manning + t * d, case.z)
        else:
            ad = float(np.dot(gz, d))

            def at(t):
                return run_loss(case.manning, case.z + t * d)
        scale = max(abs(ad), 1e-3 * loss)
        smooth = []
        for sgn in (1.0, -1.0):
            q = [(at(sgn * h) - f0) / (sgn * h) for h in (eps, eps / 2,
                                                          eps / 4)]
            r1, r2 = 2 * q[1] - q[0], 2 * q[2] - q[1]
            if abs(r1 - r2) <= 1e-7 * scale:
                smooth.append(r2)
        if smooth:
            err = min(abs(ad - v) for v in smooth) / scale
            worst = max(worst, err)
            checked += 1
            assert err <= 1e-6, (k, err)
        say(f"  direction {k}: {len(smooth)} smooth side(s)")
    f.close()
    say(f"  {checked} of 32 directions checked, worst {worst:.2e}")
    assert checked >= 24

