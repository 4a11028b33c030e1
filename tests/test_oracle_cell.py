"""Pins of the oracle's cell update (paper sec. 3.2.2, eqs. 31-37).

The semi-implicit friction step is checked against (a) the exact solution of
dq/dt = -c |q| q, which the scheme reproduces for a uniform state, and
(b) an independent evaluation of eq. 37: the friction source of eq. 5 in the
paper's primitive form, differentiated numerically at high precision, and
the 3x3 system [I - dt/2 J] dU = dt (R/A + S_f) solved by numpy.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O

G = 9.81
HDRY = 1e-6


def friction_source_eq5(h, hu, hv, m, g=G):
    """S_f of eq. 5: (0, -g h m^2 u |V| / h^(4/3), -g h m^2 v |V| / h^(4/3))
    with u = hu/h, v = hv/h, in mpmath."""
    u, v = hu / h, hv / h
    V = mp.sqrt(u * u + v * v)
    k = g * h * m * m / h ** (mp.mpf(4) / 3)
    return [mp.mpf(0), -k * u * V, -k * v * V]


def independent_update(dt, A, U, m, R):
    mp.mp.dps = 40
    U = [mp.mpf(x) for x in U]
    S = friction_source_eq5(U[0], U[1], U[2], mp.mpf(m))
    J = mp.matrix(3, 3)
    for c in range(3):
        def f(x, c=c):
            W = list(U)
            W[c] = x
            return friction_source_eq5(W[0], W[1], W[2], mp.mpf(m))
        for r in range(3):
            J[r, c] = mp.diff(lambda x: f(x)[r], U[c])
    M = mp.eye(3) - mp.mpf(dt) / 2 * J
    b = mp.matrix([mp.mpf(dt) * (mp.mpf(R[k]) / A + S[k]) for k in range(3)])
    dU = mp.lu_solve(M, b)
    return np.array([float(U[k] + dU[k]) for k in range(3)])


@pytest.mark.parametrize("seed", range(6))
def test_semi_implicit_update_matches_independent_solve(seed):
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.05, 3.0)
    U = [h, rng.normal(0, 1.5), rng.normal(0, 1.5)]
    m = rng.uniform(0.01, 0.08)
    R = rng.normal(0, 0.5, 3)
    A, dt = rng.uniform(0.5, 3.0), rng.uniform(0.01, 0.3)
    out, clamp = O.cell_update(dt, A, U, m, R)
    ref = independent_update(dt, A, U, m, R)
    assert clamp == 0.0
    assert np.max(np.abs(out - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())


def test_uniform_state_decays_exactly():
    """No net flux: 1/|q|_{n+1} = 1/|q|_n + c dt with c = g m^2 h^(-7/3),
    the exact solution of dq/dt = -c |q| q over the step, and q keeps its
    direction."""
    h, q0, m = 0.8, np.array([1.1, -0.7]), 0.035
    c = G * m * m * h ** (-7.0 / 3.0)
    dt = 0.25
    out, _ = O.cell_update(dt, 1.0, [h, *q0], m, [0.0, 0.0, 0.0])
    qn = np.hypot(*q0)
    exact = q0 / (1.0 + c * dt * qn)
    assert out[0] == h
    assert np.max(np.abs(out[1:] - exact)) < 1e-15 * qn


def test_no_friction_is_explicit_euler():
    out, _ = O.cell_update(0.1, 2.0, [1.0, 0.3, 0.2], 0.0, [0.4, -0.2, 0.6])
    assert np.allclose(out, [1.02, 0.29, 0.23], rtol=0, atol=1e-16)


def test_negative_depth_is_clamped_with_ledger():
    out, clamp = O.cell_update(1.0, 2.0, [0.1, 0.5, 0.5], 0.03,
                               [-0.4, 0.0, 0.0])
    assert out[0] == 0.0 and out[1] == 0.0 and out[2] == 0.0
    assert abs(clamp - 2.0 * 0.1) < 1e-16


def test_thin_film_loses_momentum():
    out, clamp = O.cell_update(0.1, 1.0, [1e-7, 1e-8, 0.0], 0.0,
                               [1e-7, 0.0, 0.0])
    assert clamp == 0.0 and out[0] > 0 and out[1] == 0.0 and out[2] == 0.0
