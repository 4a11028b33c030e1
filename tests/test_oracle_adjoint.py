"""Pins of the adjoint oracle (oracle/adjoint.py): its step equals the C
oracle's step, and its gradients of the gauge misfit equal central finite
differences of the C oracle's frozen-schedule runs."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import adjoint as A


def cfl_schedule(case, n):
    o = O.Oracle(case)
    dts = []
    for _ in range(n):
        o.run(1)
        dts.append(o.clock()["last_dt"])
    return np.array(dts), o


def cases():
    tr = W.dam_break_canal(nx=40, ny=6, lx=40.0, ly=6.0, h_left=1.0,
                           h_right=0.4)
    tr.hu = np.full(tr.n_cells, 0.2)
    tr.bc = {2: (W.BC_TRANSMISSIVE, 0.0), 4: (W.BC_FIXED_DEPTH, 0.9)}
    return [W.dam_break_canal(nx=40, ny=8, lx=40.0, ly=8.0),
            W.bumps_canal(nx=40, ny=14, lx=30.0, ly=10.0, x_dam=15.0),
            W.river(n_target=6_000, workers=1),
            tr]


@pytest.mark.parametrize("k", range(4))
def test_torch_step_equals_the_c_oracle(k):
    case = cases()[k]
    dts, o = cfl_schedule(case, 25)
    _, h = A.gauge_misfit(case, dts, [0], [0.0], grad=False)
    ho = o.state()[0]
    assert np.max(np.abs(h - ho)) <= 1e-13 * max(1.0, np.max(np.abs(ho)))


def misfit_problem(case, n_steps, n_gauges=64, seed=5):
    """Gauges on wet cells; the target is the run with a perturbed Manning
    field (both seeded)."""
    rng = np.random.default_rng(seed)
    wet = np.flatnonzero(case.h > 0.05)
    gauges = rng.choice(wet, size=min(n_gauges, wet.size), replace=False)
    dts, _ = cfl_schedule(case, n_steps)
    tgt_case = case.copy()
    tgt_case.manning = case.manning * (1.0 + 0.2 * rng.uniform(-1, 1,
                                                               case.n_cells))
    o = O.Oracle(tgt_case)
    o.run_dt(dts)
    return gauges, o.state()[0][gauges], dts


def c_loss(case, dts, gauges, target, m=None, z=None):
    c = case.copy()
    if m is not None:
        c.manning = m
    if z is not None:
        c.z = z
    o = O.Oracle(c)
    o.run_dt(dts)
    h = o.state()[0]
    return float(np.sum((h[gauges] - target) ** 2))


def smooth_directions(case, n, seed):
    """Seeded smooth fields over the cell centroids (a few low Fourier
    modes): perturbations along them keep neighbouring bed levels in order,
    away from the kinks of the reconstruction's max."""
    rng = np.random.default_rng(seed)
    c = case.xy[case.tri].mean(axis=1)
    span = c.max(axis=0) - c.min(axis=0)
    x = (c - c.min(axis=0)) / span
    out = []
    for _ in range(n):
        d = np.zeros(case.n_cells)
        for _ in range(4):
            kx, ky = rng.integers(1, 4, 2)
            px, py = rng.uniform(0, 2 * np.pi, 2)
            d += rng.standard_normal() * np.sin(2 * np.pi * kx * x[:, 0] + px
                                                ) * np.cos(2 * np.pi * ky *
                                                           x[:, 1] + py)
        out.append(d)
    return out


def one_sided_estimates(loss_at, f0, eps):
    """Derivative estimates of a piecewise smooth loss along a direction
    from runs at t = +-eps, +-eps/2, +-eps/4: on each side the Richardson
    values 2 D(h/2) - D(h) of the one-sided quotients D(h) = (L(s h) - f0)
    / (s h) at h = eps and eps/2. A side is smooth when its two values
    agree; a branch switch of the scheme (wet/dry threshold, wave-speed
    case, the reconstruction's max, the positivity clamp) inside the
    stencil breaks that agreement. Returns [(value, spread)] per side."""
    out = []
    for s in (1.0, -1.0):
        d = [(loss_at(s * h) - f0) / (s * h) for h in (eps, eps / 2, eps / 4)]
        r1, r2 = 2 * d[1] - d[0], 2 * d[2] - d[1]
        out.append((r2, abs(r1 - r2)))
    return out


def test_manning_gradient_matches_central_differences():
    """Manning acts smoothly on wet cells: central differences agree with
    the adjoint on every seeded direction."""
    case = W.river(n_target=6_000, workers=1)
    gauges, target, dts = misfit_problem(case, 30)
    loss, gm, gz = A.gauge_misfit(case, dts, gauges, target)
    assert loss > 0
    # the misfit is a sum of squared small differences: the relative
    # rounding of the two implementations (cbrt) is amplified
    assert abs(loss - c_loss(case, dts, gauges, target)) <= 1e-9 * loss
    wet = case.h > 0.1
    eps = 1e-6
    for d in smooth_directions(case, 4, seed=7):
        fd = (c_loss(case, dts, gauges, target, m=case.manning + eps * d * wet)
              - c_loss(case, dts, gauges, target,
                       m=case.manning - eps * d * wet)) / (2 * eps)
        ad = float(np.dot(gm, d * wet))
        assert abs(ad - fd) <= 1e-6 * max(abs(fd), 1e-3 * loss)


def test_bed_gradient_matches_one_sided_differences():
    """The bed also enters the reconstruction's max and the wet/dry
    thresholds, whose branch switches lie densely around the base state: a
    central difference straddles one in most directions (and, for a tie at
    the base state, measures the mean of the two one-sided slopes). The
    adjoint differentiates the branches taken at the base state, so it
    must equal the one-sided derivative of a side on which the loss is
    smooth (two Richardson values agreeing to 1e-7), to 1e-6. Directions
    with a branch switch within the stencil on both sides are skipped,
    at most one of four."""
    case = W.river(n_target=6_000, workers=1)
    gauges, target, dts = misfit_problem(case, 30)
    loss, gm, gz = A.gauge_misfit(case, dts, gauges, target)
    f0 = c_loss(case, dts, gauges, target)
    checked = 0
    for d in smooth_directions(case, 4, seed=7):
        ad = float(np.dot(gz, d))
        scale = max(abs(ad), 1e-3 * loss)
        est = one_sided_estimates(
            lambda t: c_loss(case, dts, gauges, target, z=case.z + t * d),
            f0, 1e-6)
        smooth = [v for v, spread in est if spread <= 1e-7 * scale]
        if not smooth:
            continue
        checked += 1
        assert min(abs(ad - v) for v in smooth) <= 1e-6 * scale, est
    assert checked >= 3


def test_frictionless_canal_has_zero_manning_gradient():
    """At m = 0 the Manning gradient vanishes identically: the friction
    coefficient g m^2 / h^(7/3) is quadratic in m; the bed gradient does
    not."""
    case = W.dam_break_canal(nx=30, ny=6, lx=30.0, ly=6.0)
    gauges, target, dts = misfit_problem(case, 15, n_gauges=10)
    _, gm, gz = A.gauge_misfit(case, dts, gauges, target + 0.01)
    assert np.all(gm == 0.0)
    assert np.any(gz != 0.0)
