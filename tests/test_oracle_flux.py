"""Pins of the oracle's edge numerics (paper sec. 3.1-3.2.1, eqs. 12-30).

Each check compares the oracle with something other than itself: the exact
shallow-water Riemann solution, Rankine-Hugoniot shock speeds, closed forms,
or invariants the method must have (consistency, mirror symmetry, rotational
invariance, well-balancing). No formula of the oracle is retyped here.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O
from riemann_exact import (godunov_flux, shock_speed_left, shock_speed_right,
                           star_state)

G = 9.81
HDRY = 1e-6


def phys(h, u, v, g=G):
    return np.array([h * u, h * u * u + 0.5 * g * h * h, h * u * v])


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def random_states(n, seed, dry_frac=0.0):
    rng = np.random.default_rng(seed)
    hL = rng.uniform(0.05, 5.0, n)
    hR = rng.uniform(0.05, 5.0, n)
    if dry_frac:
        hL[rng.random(n) < dry_frac] = 0.0
        hR[rng.random(n) < dry_frac] = 0.0
    uL, uR = rng.normal(0, 2, n), rng.normal(0, 2, n)
    vL, vR = rng.normal(0, 2, n), rng.normal(0, 2, n)
    return hL, uL, vL, hR, uR, vR


# ---------------------------------------------------------------- HLLC flux

def test_consistency_equal_states():
    """G~(U, U) = G(U) (eq. 17 with U_L = U_R)."""
    hL, uL, vL, *_ = random_states(500, 1)
    for h, u, v in zip(hL, uL, vL):
        assert rel(O.hllc(h, u, v, h, u, v), phys(h, u, v)) < 1e-14


def test_mirror_symmetry_including_dry_sides():
    """Reflecting the problem (swap sides, flip the normal velocity) flips the
    mass and tangential fluxes and keeps the normal-momentum flux; this pins
    the right-dry line of eq. 26 against the left-dry one."""
    hL, uL, vL, hR, uR, vR = random_states(2000, 2, dry_frac=0.3)
    worst = 0.0
    for a in zip(hL, uL, vL, hR, uR, vR):
        G1 = O.hllc(*a)
        h1, u1, v1, h2, u2, v2 = a
        G2 = O.hllc(h2, -u2, v2, h1, -u1, v1)
        scale = max(np.abs(G1).max(), 1.0)
        worst = max(worst, abs(G1[0] + G2[0]) / scale,
                    abs(G1[1] - G2[1]) / scale, abs(G1[2] + G2[2]) / scale)
    assert worst < 1e-13


def test_both_dry_is_zero():
    assert np.all(O.hllc(0.0, 1.0, 1.0, 5e-7, -1.0, 2.0) == 0.0)


def test_supersonic_upwind():
    """S_L >= 0 gives the left physical flux, S_R <= 0 the right one."""
    G1 = O.hllc(1.0, 8.0, 0.3, 0.8, 7.0, -0.2)
    assert rel(G1, phys(1.0, 8.0, 0.3)) < 1e-15
    G2 = O.hllc(1.0, -8.0, 0.3, 0.8, -7.0, -0.2)
    assert rel(G2, phys(0.8, -7.0, -0.2)) < 1e-15


@pytest.mark.parametrize("u", [0.7, -0.7, 3.5, -3.5])
def test_contact_carries_upwind_tangential_velocity(u):
    """Pure contact (equal depth and normal velocity, jump in the tangential
    velocity): the exact Godunov flux of the passive tangential momentum is
    taken from the side the contact comes from (eq. 24, upwind reading)."""
    h = 1.3
    Gx = O.hllc(h, u, 0.9, h, u, -0.4)
    Ge = [float(x) for x in godunov_flux(h, u, 0.9, h, u, -0.4)]
    assert rel(Gx, Ge) < 1e-13


# ---------------------------------------------------- star depth (eqs. 21-23)

@pytest.mark.parametrize("h,w", [(1.0, 0.5), (2.0, 3.0), (0.3, 0.1),
                                 (5.0, 7.0)])
def test_two_rarefaction_symmetric_is_exact(h, w):
    """Symmetric expansion u_L = -w, u_R = w: the exact star depth is
    (sqrt(g h) - w/2)^2 / g from the Riemann invariants u +- 2a; the
    rarefaction estimate (eq. 22) must return it."""
    h0, hs, br = O.star_depth(h, -w, h, w)
    assert br == 0
    exact = (math.sqrt(G * h) - w / 2) ** 2 / G
    assert abs(hs - exact) <= 1e-14 * exact


def test_two_rarefaction_asymmetric_matches_exact_solver():
    """Whenever the exact solution has two rarefactions and eq. 21 selects
    the rarefaction branch, eq. 22 is exact."""
    rng = np.random.default_rng(3)
    checked = 0
    while checked < 40:
        hL, hR = rng.uniform(0.1, 4.0, 2)
        uL, uR = -rng.uniform(0.0, 2.0), rng.uniform(0.0, 2.0)
        hs_ex, _ = star_state(hL, uL, hR, uR)
        if not (hs_ex < min(hL, hR) and hs_ex > 0):
            continue
        h0, hs, br = O.star_depth(hL, uL, hR, uR)
        if br != 0:
            continue
        assert abs(hs - float(hs_ex)) <= 1e-13 * float(hs_ex)
        checked += 1


def test_vacuum_gives_zero_star_depth():
    """u_R - u_L > 2(a_L + a_R) opens a dry gap: h* = 0 (vacuum reading of
    eq. 22), and the mass flux of the symmetric problem vanishes."""
    h0, hs, br = O.star_depth(1.0, -8.0, 1.0, 8.0)
    assert br == 0 and hs == 0.0
    G1 = O.hllc(1.0, -8.0, 0.0, 1.0, 8.0, 0.0)
    assert abs(G1[0]) < 1e-14


def _two_shock_data(hL, hR, hs, g=G):
    """Velocity jump u_L - u_R for which the exact solution is two shocks
    with star depth hs (shock relations of both waves)."""
    fL = (hs - hL) * math.sqrt(g * (hs + hL) / (2 * hs * hL))
    fR = (hs - hR) * math.sqrt(g * (hs + hR) / (2 * hs * hR))
    return fL + fR


def test_two_shock_estimate_converges_second_order():
    """For two-shock data of amplitude d the shock estimate (eqs. 21, 23)
    approaches the exact star depth. Eq. 23 is exact at its own fixed point,
    so its error is O(d) times that of the seed h0 of eq. 21. With the
    coefficient 1/4 printed in eq. 21 the seed is first-order (the exact
    linearisation has 1/2), so the estimate converges like d^2; a sign or
    index mistake in eq. 23 would leave an O(d) error."""
    errs = []
    for d in [0.2, 0.1, 0.05, 0.025]:
        hL, hR = 1.0, 1.0 + 0.3 * d
        hs = 1.0 + d + 0.3 * d
        du = _two_shock_data(hL, hR, hs)
        _, est, br = O.star_depth(hL, du, hR, 0.0)
        assert br == 1
        errs.append(abs(est - hs))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(3)]
    assert min(rates) > 1.8, (errs, rates)


def test_star_depth_estimates_track_exact_solution():
    """Across random wet Riemann problems the estimate stays within 10 % of
    the exact star depth (both branches)."""
    rng = np.random.default_rng(4)
    for _ in range(200):
        hL, hR = rng.uniform(0.1, 4.0, 2)
        uL, uR = rng.normal(0, 1.0, 2)
        hs_ex, _ = star_state(hL, uL, hR, uR)
        if hs_ex == 0:
            continue
        _, hs, _ = O.star_depth(hL, uL, hR, uR)
        assert abs(hs - float(hs_ex)) <= 0.1 * float(hs_ex)


# ---------------------------------------------------- wave speeds (eqs. 19-20)

@pytest.mark.parametrize("hL,uL,hs", [(1.0, 0.0, 1.7), (0.4, 2.0, 2.5),
                                      (3.0, -1.0, 3.01)])
def test_left_shock_speed_is_rankine_hugoniot(hL, uL, hs):
    """With the exact star depth, S_L of eqs. 19-20 is the exact speed of a
    left shock (mass Rankine-Hugoniot); this pins the /h_k reading of eq.
    20."""
    SL, _ = O.wave_speeds_given_hs(hL, uL, 1.0, 0.0, hs)
    assert abs(SL - float(shock_speed_left(hL, uL, hs))) < 1e-13 * (1 + abs(SL))


@pytest.mark.parametrize("hR,uR,hs", [(1.0, 0.0, 1.7), (0.4, -2.0, 2.5)])
def test_right_shock_speed_is_rankine_hugoniot(hR, uR, hs):
    _, SR = O.wave_speeds_given_hs(1.0, 0.0, hR, uR, hs)
    assert abs(SR - float(shock_speed_right(hR, uR, hs))) < 1e-13 * (1 + abs(SR))


def test_rarefaction_heads_are_characteristic_speeds():
    """For h* <= h_k the estimate is the rarefaction head u_k -+ a_k."""
    SL, SR = O.wave_speeds_given_hs(2.0, 0.5, 3.0, -0.25, 1.0)
    assert SL == 0.5 - math.sqrt(G * 2.0)
    assert SR == -0.25 + math.sqrt(G * 3.0)


def test_contact_speed_equals_velocity_for_uniform_normal_flow():
    """Equal depth and normal velocity: S* (eq. 25) is that velocity."""
    for u in [-1.3, 0.0, 0.4, 2.2]:
        _, _, Ss = O.wave_speeds(1.7, u, 1.7, u)
        assert abs(Ss - u) < 1e-14 * max(1.0, abs(u))


def test_dry_bed_front_speeds():
    """A dry side: the front moves at u + 2a into the dry region (Ritter),
    and S* sits on the front (eq. 26)."""
    SL, SR, Ss = O.wave_speeds(2.0, 0.3, 0.0, 0.0)
    a = math.sqrt(G * 2.0)
    assert SR == 0.3 + 2 * a and Ss == SR and SL == 0.3 - a
    SL, SR, Ss = O.wave_speeds(0.0, 0.0, 2.0, -0.3)
    assert SL == -0.3 - 2 * a and Ss == SL and SR == -0.3 + a


def test_dry_bed_flux_direction():
    """Dam break onto a dry bed from rest: water and momentum flow towards
    the dry side, and nothing flows when the wet side sits still against a
    dry bed that is higher (handled by the reconstruction, not here)."""
    Gx = O.hllc(1.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    assert Gx[0] > 0 and Gx[1] > 0 and Gx[2] == 0
    Gm = O.hllc(0.0, 0.0, 0.0, 1.0, 0.0, 0.0)
    assert Gm[0] == -Gx[0] and Gm[1] == Gx[1]


# ---------------------------------------------- edge contributions (eqs. 12, 28-30)

def _rot(t):
    return np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])


def test_rotational_invariance_of_edge():
    """Rotating the normal and both velocities by theta rotates the momentum
    contributions and leaves the mass contribution unchanged (eq. 12)."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        hi, hj = rng.uniform(0.1, 3.0, 2)
        qi, qj = rng.normal(0, 2, 2), rng.normal(0, 2, 2)
        zi, zj = rng.uniform(0, 1, 2)
        t0 = rng.uniform(0, 2 * math.pi)
        n = np.array([math.cos(t0), math.sin(t0)])
        L = rng.uniform(0.5, 2.0)
        cl, cr = O.interior_edge([hi, *qi], zi, [hj, *qj], zj, n, L)
        th = rng.uniform(0, 2 * math.pi)
        R = _rot(th)
        cl2, cr2 = O.interior_edge([hi, *(R @ qi)], zi, [hj, *(R @ qj)], zj,
                                   R @ n, L)
        s = max(np.abs(cl).max(), np.abs(cr).max(), 1.0)
        assert abs(cl2[0] - cl[0]) < 1e-12 * s
        assert np.abs(cl2[1:] - R @ cl[1:]).max() < 1e-12 * s
        assert np.abs(cr2[1:] - R @ cr[1:]).max() < 1e-12 * s


def test_edge_along_x_is_one_dimensional_flux():
    """n = (1, 0): the mass and x-momentum contributions are those of the
    1-D problem in x, and the y-momentum one is the tangential flux."""
    Ui, Uj = [1.2, 0.6, 0.24], [0.7, -0.35, 0.14]
    cl, cr = O.interior_edge(Ui, 0.0, Uj, 0.0, [1.0, 0.0], 2.0)
    G1 = O.hllc(1.2, 0.5, 0.2, 0.7, -0.5, 0.2)
    assert rel(-cl, 2.0 * G1) < 1e-15 and rel(cr, 2.0 * G1) < 1e-15


@pytest.mark.parametrize("eta,zi,zj", [(1.0, 0.2, 0.5), (1.0, 0.7, 0.1),
                                       (0.3, 0.1, 0.5), (0.3, 0.6, 0.0)])
def test_lake_at_rest_edge_is_hydrostatic(eta, zi, zj):
    """Still water with a flat surface (a cell may be dry above it): each
    side receives exactly the hydrostatic push -+L (g/2) h^2 n of its own
    depth, whatever the bed step. Summed over a closed cell this vanishes,
    which is the well-balanced property the reading of eq. 30 (factor g/2)
    and of eq. 37 (reconstructed states) must deliver."""
    hi, hj = max(0.0, eta - zi), max(0.0, eta - zj)
    n = np.array([0.6, 0.8])
    L = 1.7
    cl, cr = O.interior_edge([hi, 0, 0], zi, [hj, 0, 0], zj, n, L)
    pi, pj = 0.5 * G * hi * hi * L, 0.5 * G * hj * hj * L
    assert abs(cl[0]) < 1e-15 and abs(cr[0]) < 1e-15
    assert np.abs(cl[1:] + pi * n).max() < 1e-14 * max(pi, 1)
    assert np.abs(cr[1:] - pj * n).max() < 1e-14 * max(pj, 1)


def test_flat_bed_edge_is_conservative():
    """On a flat bed the two sides receive opposite contributions."""
    rng = np.random.default_rng(6)
    for _ in range(100):
        Ui = [rng.uniform(0, 2), *rng.normal(0, 1, 2)]
        Uj = [rng.uniform(0, 2), *rng.normal(0, 1, 2)]
        cl, cr = O.interior_edge(Ui, 0.3, Uj, 0.3, [0.8, -0.6], 1.1)
        assert np.all(cl == -cr)


# ------------------------------------------------------------ boundary edges

def test_wall_flux_is_hydrostatic_pressure():
    n = np.array([0.0, -1.0])
    cl = O.boundary_edge(0, 0.0, 0.0, [2.0, 0.3, -0.4], 0.5, n, 3.0)
    assert cl[0] == 0.0
    assert np.allclose(cl[1:], -3.0 * 0.5 * G * 4.0 * n, rtol=1e-15)


def test_transmissive_equals_interior_with_equal_states():
    """U_R = U_L (sec. 3.1): the same as an interior edge between two equal
    cells on a flat bed."""
    U = [1.1, 0.4, -0.9]
    n = np.array([0.28, 0.96])
    cl = O.boundary_edge(1, 0.0, 0.0, U, 0.0, n, 1.5)
    cl2, _ = O.interior_edge(U, 0.0, U, 0.0, n, 1.5)
    assert rel(cl, cl2) < 1e-14


def test_inflow_with_matching_state_equals_transmissive():
    """If the cell already carries the inflow discharge q along -n with no
    tangential velocity, the inflow flux equals the transmissive one."""
    h, q = 1.4, 2.5
    n = np.array([-1.0, 0.0])
    U = [h, -q * n[0], -q * n[1]]
    ci = O.boundary_edge(2, 0.0, q, U, 0.0, n, 1.0)
    ct = O.boundary_edge(1, 0.0, 0.0, U, 0.0, n, 1.0)
    assert rel(ci, ct) < 1e-15
    assert ci[0] == q


def test_fixed_depth_with_cell_depth_equals_transmissive():
    U = [0.9, 0.2, 0.1]
    n = np.array([1.0, 0.0])
    cf = O.boundary_edge(3, 0.9, 0.0, U, 0.0, n, 1.0)
    ct = O.boundary_edge(1, 0.0, 0.0, U, 0.0, n, 1.0)
    assert rel(cf, ct) < 1e-14
    cs = O.boundary_edge(4, 0.9 + 0.25, 0.0, U, 0.25, n, 1.0)
    assert rel(cs, ct) < 1e-14


# ----------------------------------------- fixed depth / fixed stage (R16)
# The downstream level is held by a ghost cell outside the boundary edge: it
# has the prescribed depth (or the depth of the prescribed surface above the
# cell's bed) and the cell's own velocity, and the edge flux is the Riemann
# flux between the cell (inside, left of the outward normal) and the ghost.

def rotated(cl, n, L):
    """Flux (G0, G1, G2) in the edge frame from a contribution cl = -L F."""
    F0, F1, F2 = -cl[0] / L, -cl[1] / L, -cl[2] / L
    return np.array([F0, F1 * n[0] + F2 * n[1], -F1 * n[1] + F2 * n[0]])


def ghost_cases(seed, n=400):
    """Cell states with oblique velocities, ghost depths above and below."""
    rng = np.random.default_rng(seed)
    for _ in range(n):
        h = rng.uniform(0.1, 3.0)
        u, v = rng.normal(0, 1.0, 2)
        hb = h * rng.uniform(0.3, 2.5)
        th = rng.uniform(0, 2 * np.pi)
        yield h, u, v, hb, np.array([np.cos(th), np.sin(th)])


def test_fixed_depth_ghost_is_the_outer_neighbour():
    """On a flat bed the boundary edge equals, exactly, an interior edge
    whose right (outer) cell holds the ghost (h_b, h_b u, h_b v): the ghost
    sits outside, beyond the outward normal, and moves with the cell."""
    inflow = outflow = 0
    for h, u, v, hb, n in ghost_cases(11):
        L = 1.7
        cb = O.boundary_edge(3, hb, 0.0, [h, h * u, h * v], 0.4, n, L)
        ci, _ = O.interior_edge([h, h * u, h * v], 0.4,
                                [hb, hb * u, hb * v], 0.4, n, L)
        # the interior edge recovers u = (h_b u) / h_b, which may round
        assert rel(cb, ci) < 1e-14
        inflow += cb[0] > 0
        outflow += cb[0] < 0
    assert inflow > 50 and outflow > 50   # both directions exercised


def test_fixed_stage_ghost_depth_is_stage_minus_bed():
    """A fixed surface elevation s over a cell of bed z is the fixed depth
    s - z, and a stage below the bed leaves a dry ghost (depth 0)."""
    rng = np.random.default_rng(12)
    for h, u, v, hb, n in ghost_cases(13, 200):
        z = rng.uniform(-2.0, 2.0)
        U = [h, h * u, h * v]
        cs = O.boundary_edge(4, z + hb, 0.0, U, z, n, 1.3)
        cd = O.boundary_edge(3, hb, 0.0, U, z, n, 1.3)
        assert rel(cs, cd) < 1e-14
        cdry = O.boundary_edge(4, z - 0.5, 0.0, U, z, n, 1.3)
        assert np.array_equal(cdry, O.boundary_edge(3, 0.0, 0.0, U, z, n,
                                                    1.3))
        ci, _ = O.interior_edge(U, z, [0.0, 0.0, 0.0], z, n, 1.3)
        assert np.array_equal(cdry, ci)


@pytest.mark.parametrize("kind", [3, 4])
def test_deeper_ghost_fills_and_shallower_drains_a_still_cell(kind):
    """Water at rest next to a higher held level flows in, next to a lower
    one flows out. For mild level differences the rate is that of the exact
    Godunov flux of the dam break between the two (HLLC tracks it to 5 %
    there; for strong ones only the direction is checked)."""
    n = np.array([0.6, -0.8])
    L = 2.0
    z = 0.3
    cases = [(1.0, 1.2, True), (1.0, 0.8, True), (1.0, 1.05, True),
             (2.0, 1.7, True), (0.5, 0.6, True), (0.4, 2.0, False),
             (1.5, 0.2, False), (0.8, 0.0, False)]
    for h, hb, mild in cases:
        value = hb if kind == 3 else z + hb
        cl = O.boundary_edge(kind, value, 0.0, [h, 0.0, 0.0], z, n, L)
        G = rotated(cl, n, L)
        # outward mass flux: negative (inflow) iff the ghost is deeper
        assert (G[0] < 0) == (hb > h) and G[0] != 0.0
        if mild:
            Ge = [float(x) for x in godunov_flux(h, 0.0, 0.0, hb, 0.0, 0.0)]
            assert abs(G[0] - Ge[0]) <= 0.05 * abs(Ge[0])
            assert abs(G[1] - Ge[1]) <= 0.05 * abs(Ge[1])


@pytest.mark.parametrize("kind", [3, 4])
def test_ghost_carries_the_cell_tangential_velocity(kind):
    """Both sides of the held-level Riemann problem move along the edge with
    the cell's tangential velocity u_t, so whatever the direction of the
    flow the tangential momentum flux is the mass flux times u_t (exactly so
    in the Godunov flux, where u_t is carried by the contact)."""
    seen_in = 0
    for h, u, v, hb, n in ghost_cases(14):
        z = 0.2
        value = hb if kind == 3 else z + hb
        cl = O.boundary_edge(kind, value, 0.0, [h, h * u, h * v], z, n, 1.0)
        G = rotated(cl, n, 1.0)
        ut = -u * n[1] + v * n[0]
        assert abs(G[2] - G[0] * ut) <= 1e-13 * max(1.0, abs(G[0] * ut))
        seen_in += G[0] < -1e-3 and abs(ut) > 0.1
    assert seen_in > 30
