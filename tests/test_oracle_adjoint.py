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


@pytest.mark.parametrize("which", ["manning", "z"])
def test_gradients_match_central_differences(which):
    case = W.river(n_target=6_000, workers=1)
    gauges, target, dts = misfit_problem(case, 30)
    loss, gm, gz = A.gauge_misfit(case, dts, gauges, target)
    assert loss > 0
    # the misfit is a sum of squared small differences: the relative
    # rounding of the two implementations (cbrt) is amplified
    assert abs(loss - c_loss(case, dts, gauges, target)) <= 1e-9 * loss
    # Manning acts smoothly on wet cells; the bed also enters the
    # reconstruction's max and the wet/dry thresholds, whose kinks a
    # finite-difference stencil crosses now and then: the bed takes the
    # better of two step sizes and a looser bar
    wet = case.h > 0.1
    for d in smooth_directions(case, 4, seed=7):
        errs = []
        for eps in ((1e-6,) if which == "manning" else (1e-6, 1e-7)):
            if which == "manning":
                args_p = dict(m=case.manning + eps * d * wet)
                args_m = dict(m=case.manning - eps * d * wet)
                dd = float(np.dot(gm, d * wet))
            else:
                args_p = dict(z=case.z + eps * d)
                args_m = dict(z=case.z - eps * d)
                dd = float(np.dot(gz, d))
            fd = (c_loss(case, dts, gauges, target, **args_p) -
                  c_loss(case, dts, gauges, target, **args_m)) / (2 * eps)
            errs.append(abs(dd - fd) / max(abs(fd), 1e-3 * loss))
        assert min(errs) <= (1e-6 if which == "manning" else 1e-5), errs


def test_frictionless_canal_has_zero_manning_gradient():
    """At m = 0 the Manning gradient vanishes identically: the friction
    coefficient g m^2 / h^(7/3) is quadratic in m; the bed gradient does
    not."""
    case = W.dam_break_canal(nx=30, ny=6, lx=30.0, ly=6.0)
    gauges, target, dts = misfit_problem(case, 15, n_gauges=10)
    _, gm, gz = A.gauge_misfit(case, dts, gauges, target + 0.01)
    assert np.all(gm == 0.0)
    assert np.any(gz != 0.0)
