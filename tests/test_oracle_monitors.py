"""Pins of the oracle's monitors: the outflow / inflow rates per boundary tag
(sec. 5.3.2) and the flood envelope (maximum depth and first wetting time,
from which the flood lines of sec. 6.4.3 are drawn).

Each pin checks the monitors against something other than their own code:
boundary-condition values (an inflow tag passes exactly -Q, a wall nothing),
the water balance with the positivity ledger, the normal flux of the state
for a transmissive edge, and the trajectory recorded step by step.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def test_closed_canal_has_no_boundary_flow():
    case = W.dam_break_canal()
    o = O.Oracle(case)
    o.run(40)
    for tag in (0, 1, 2, 3, 4):
        assert o.discharge(tag) == (0.0, 0.0)


def test_inflow_tag_passes_minus_q_and_balance_closes():
    case = W.river(n_target=20_000, workers=1)
    q_in = case.bc[1][1]
    o = O.Oracle(case)
    m0 = o.mass()
    led0 = o.clock()["ledger"]
    t_total = 0.0
    for _ in range(30):
        o.run(1)
        rate, vol = o.discharge(1)
        # q = Q / (tag length) on every inflow edge, so sum L q = Q
        assert abs(rate + q_in) <= 1e-12 * q_in
        t_total += o.clock()["last_dt"]
        assert abs(vol + q_in * t_total) <= 1e-11 * q_in * t_total
    out = sum(o.discharge(tag)[1] for tag in (0, 1, 2))
    dm = o.mass() - m0
    led = o.clock()["ledger"] - led0
    scale = q_in * t_total
    assert abs(dm - (-out + led)) <= 1e-9 * scale, (dm, out, led)


def test_transmissive_rate_is_the_normal_flux_of_the_state():
    case = W.dam_break_canal(nx=60, ny=6, lx=60.0, ly=6.0, h_left=1.0,
                             h_right=0.4)
    case.hu = np.full(case.n_cells, 0.3)     # flow towards the east end
    case.bc = {2: (W.BC_TRANSMISSIVE, 0.0)}
    o = O.Oracle(case)
    e = o.edges()
    east = (e["right"] < 0) & (e["tag"] == 2)
    for _ in range(5):
        h, hu, hv = o.state()
        cells = e["left"][east]
        nx, ny, ln = e["nx"][east], e["ny"][east], e["len"][east]
        # outward mass flux h u_n = hu n_x + hv n_y of the cell beside it
        expect = math.fsum(ln * (hu[cells] * nx + hv[cells] * ny))
        o.run(1)
        rate, _ = o.discharge(2)
        assert abs(rate - expect) <= 1e-12 * abs(expect)
        assert rate > 0.0


def test_envelope_matches_the_recorded_trajectory():
    case = W.bumps_canal(nx=40, ny=14, lx=30.0, ly=10.0, x_dam=15.0)
    o = O.Oracle(case)
    h0 = o.state()[0]
    hmax = h0.copy()
    twet = np.where(h0 > case.h_dry, 0.0, np.inf)
    for _ in range(60):
        o.run(1)
        h = o.state()[0]
        t = o.clock()["t"]
        newly = np.isinf(twet) & (h > case.h_dry)
        twet[newly] = t
        hmax = np.maximum(hmax, h)
    om, ot = o.envelope()
    assert np.array_equal(om, hmax)
    assert np.array_equal(ot, twet)
    assert np.any(np.isfinite(twet) & (twet > 0))    # the front advanced
    assert np.any(np.isinf(twet))                     # not everywhere yet


def test_setting_the_state_resets_the_monitors():
    case = W.river(n_target=20_000, workers=1)
    o = O.Oracle(case)
    o.run(10)
    assert o.discharge(1)[1] != 0.0
    h, hu, hv = o.state()
    o.set_state(h, hu, hv)
    assert o.discharge(1) == (0.0, 0.0)
    hm, tw = o.envelope()
    assert np.array_equal(hm, h)
    t = o.clock()["t"]
    assert np.array_equal(tw, np.where(h > case.h_dry, t, np.inf))
