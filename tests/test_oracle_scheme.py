"""Whole-scheme pins of the oracle: closed-form solutions and invariants.

* Stoker's dam break (exact Riemann solution, two wet states) on the
  100 m x 20 m canal, and convergence of the error under refinement.
* Ritter's dam break onto a dry bed.
* Lake at rest over bumps with dry bump tops (well-balancing).
* Mass: exact in a closed basin up to the positivity ledger; inflow Q adds
  exactly Q t.
* Exact Manning decay of a uniform flow.
* Rotational invariance, cell-permutation invariance and thread-count
  independence of the whole step.
* Mesh validation errors.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from riemann_exact import profile, star_state

G = 9.81


def run(case, steps=None, t_end=None, threads=0):
    o = O.Oracle(case, threads=threads)
    o.run(case.steps if steps is None else steps,
          case.t_end if t_end is None else t_end)
    return o


def mass(o):
    area, _, _ = o.geometry()
    h, _, _ = o.state()
    return math.fsum(area * h)


# ------------------------------------------------------------------ Stoker

def centreline(case, h, y0, y1):
    cen = case.centroids()
    m = (cen[:, 1] > y0) & (cen[:, 1] < y1)
    idx = np.argsort(cen[m, 0], kind="stable")
    return cen[m, 0][idx], h[m][idx]


def stoker_profile(x, t, hl, hr, x0):
    return profile(hl, 0.0, hr, 0.0, (np.asarray(x) - x0) / t)[0]


def test_stoker_dam_break_plateau_and_shock():
    case = W.dam_break_canal()
    o = run(case)
    assert o.clock()["t"] == 5.0
    h, _, _ = o.state()
    x, hc = centreline(case, h, 9.0, 11.0)
    hm, um = star_state(1.0, 0.0, 0.5, 0.0)
    hm = float(hm)
    assert abs(hm - 0.726920446) < 1e-8
    plateau = hc[(x > 45) & (x < 60)]
    assert np.max(np.abs(plateau - hm)) < 0.01 * hm
    # shock at x0 + S t: the centreline depth crosses the mid-level there
    S = 2.9579181201875
    mid = 0.5 * (hm + 0.5)
    xs = x[np.argmax((hc < mid) & (x > 55))]
    assert abs(xs - (50 + 5 * S)) <= 2.0
    # well ahead of the rarefaction head (x = 34.3) the water is undisturbed
    # but for the first-order scheme's numerical diffusion
    assert np.all(np.abs(hc[x < 25] - 1.0) < 1e-3)


def test_stoker_error_falls_under_refinement():
    errs = []
    for k in (1, 2, 4):
        case = W.dam_break_canal(nx=100 * k, ny=20 * k)
        case.t_end = 2.0
        o = run(case, threads=0)
        h, _, _ = o.state()
        x, hc = centreline(case, h, 9.0, 11.0)
        ex = stoker_profile(x, 2.0, 1.0, 0.5, 50.0)
        errs.append(np.mean(np.abs(hc - ex)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.6 * errs[0]


# ------------------------------------------------------------------ Ritter

def test_ritter_dry_bed_dam_break():
    case = W.dam_break_canal(nx=400, ny=16, lx=100.0, ly=4.0, h_right=0.0,
                             t_end=2.0)
    o = run(case)
    h, hu, _ = o.state()
    x, hc = centreline(case, h, 1.5, 2.5)
    c0 = math.sqrt(G)
    t = 2.0
    xi = (x - 50.0) / t
    fan = (xi > -0.7 * c0) & (xi < 1.0 * c0)
    exact = (2 * c0 - xi[fan]) ** 2 / (9 * G)
    assert np.mean(np.abs(hc[fan] - exact)) < 0.01
    # at the dam the exact depth is 4/9 h0 at all times; the dam is the sonic
    # point of the fan, where first-order Riemann-solver schemes carry their
    # largest (few per cent) error
    at_dam = np.abs(x - 50.0) < 0.5
    ex_dam = (2 * c0 - xi[at_dam]) ** 2 / (9 * G)
    assert abs((2 * c0) ** 2 / (9 * G) - 4.0 / 9.0) < 1e-15
    assert np.all(np.abs(hc[at_dam] - ex_dam) < 0.03)
    # no water far beyond the exact front at 2 c0 t
    assert np.all(hc[x > 50 + 2 * c0 * t + 3.0] == 0.0)
    # water never goes negative, momentum zero where dry
    assert np.all(h >= 0) and np.all(hu[h <= case.h_dry] == 0)


# ------------------------------------------------------------ lake at rest

def test_lake_at_rest_over_bumps_with_dry_tops():
    case = W.lake_at_rest(nx=100, ny=40)
    assert np.any(case.h == 0.0) and np.any(case.h > 0.0)
    o = run(case, steps=2000)
    h, hu, hv = o.state()
    wet = h > 0
    assert np.max(np.abs(hu)) <= 1e-12 and np.max(np.abs(hv)) <= 1e-12
    assert np.max(np.abs(h[wet] + case.z[wet] - 0.12)) <= 1e-12
    assert np.all(h[~wet] == 0.0)


# ------------------------------------------------------------------- mass

def test_mass_closed_basin_dam_break():
    case = W.dam_break_canal()
    o = O.Oracle(case)
    m0 = mass(o)
    o.run(10**9, 5.0)
    assert abs(mass(o) - m0) / m0 < 1e-13


def test_mass_and_ledger_dry_bed_with_bumps():
    case = W.bumps_canal(nx=200, ny=50, steps=400)
    o = O.Oracle(case)
    m0 = mass(o)
    o.run(case.steps)
    ledger = o.clock()["ledger"]
    assert abs(mass(o) - m0 - ledger) / m0 < 1e-13


def test_inflow_adds_exactly_q_t():
    case = W.dam_break_canal(nx=40, ny=20, lx=20.0, ly=10.0, h_left=0.5,
                             h_right=0.5)
    case.bc = {4: (W.BC_INFLOW, 2.0)}        # west side
    o = O.Oracle(case)
    m0 = mass(o)
    o.run(200)
    t = o.clock()["t"]
    ledger = o.clock()["ledger"]
    assert abs(mass(o) - m0 - 2.0 * t - ledger) / m0 < 1e-12


# ------------------------------------------------------------ friction decay

def test_uniform_flow_decays_like_manning_closed_form():
    """Uniform state, transmissive boundaries, flat bed: every cell follows
    1/|q| = 1/|q0| + c t exactly, c = g m^2 h^(-7/3)."""
    case = W.dam_break_canal(nx=30, ny=10, lx=30.0, ly=10.0, h_left=0.7,
                             h_right=0.7)
    case.hu[:] = 0.9
    case.hv[:] = -0.4
    case.manning[:] = 0.04
    case.bc = {k: (W.BC_TRANSMISSIVE, 0.0) for k in (1, 2, 3, 4)}
    o = O.Oracle(case)
    o.run(150)
    t = o.clock()["t"]
    h, hu, hv = o.state()
    c = G * 0.04 ** 2 * 0.7 ** (-7.0 / 3.0)
    q0 = math.hypot(0.9, -0.4)
    q_exact = 1.0 / (1.0 / q0 + c * t)
    assert np.max(np.abs(h - 0.7)) < 1e-13
    assert np.max(np.abs(np.hypot(hu, hv) - q_exact)) < 1e-13
    assert np.max(np.abs(hu / hv - 0.9 / -0.4)) < 1e-12


# ------------------------------------------------------------- time step

def test_first_time_step_follows_inradius_rule():
    """dt = CFL * R / (sqrt(g h) + |V|) with R the inscribed radius (sec. 3.1):
    the canal's cells are right isosceles triangles with unit legs, whose
    inscribed radius is (1 + 1 - sqrt 2) / 2."""
    case = W.dam_break_canal(nx=10, ny=2, lx=10.0, ly=2.0, h_left=2.0,
                             h_right=2.0)
    case.hu[:] = 2.0 * 0.5
    case.hv[:] = 2.0 * -0.25
    o = O.Oracle(case)
    o.run(1)
    r = (2.0 - math.sqrt(2.0)) / 2.0
    s = math.sqrt(G * 2.0) + math.hypot(0.5, -0.25)
    assert abs(o.clock()["last_dt"] - 0.9 * r / s) < 1e-15


def test_last_step_lands_on_end_time():
    case = W.dam_break_canal(nx=10, ny=2, lx=10.0, ly=2.0)
    o = O.Oracle(case)
    n, t = o.run(1000, 0.3)
    assert t == 0.3 and o.clock()["t"] == 0.3 and n >= 2


# ---------------------------------------------------------------- invariance

def test_rotation_invariance_of_whole_step():
    base = W.bumps_canal(nx=60, ny=20, lx=30.0, ly=10.0, x_dam=15.0,
                         steps=40)
    base.manning[:] = 0.03
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    rot = base.copy()
    rot.xy = base.xy @ R.T
    o1 = run(base)
    o2 = run(rot)
    h1, hu1, hv1 = o1.state()
    h2, hu2, hv2 = o2.state()
    q1 = np.stack([hu1, hv1], 1) @ R.T
    assert np.max(np.abs(h1 - h2)) < 1e-11
    assert np.max(np.abs(q1[:, 0] - hu2)) < 1e-11
    assert np.max(np.abs(q1[:, 1] - hv2)) < 1e-11


def test_cell_permutation_gives_identical_bits():
    base = W.bumps_canal(nx=60, ny=20, lx=30.0, ly=10.0, x_dam=15.0,
                         steps=50)
    perm = np.random.default_rng(9).permutation(base.n_cells)
    p = base.copy()
    p.tri, p.z, p.manning = base.tri[perm], base.z[perm], base.manning[perm]
    p.h, p.hu, p.hv = base.h[perm], base.hu[perm], base.hv[perm]
    a = run(base).state()
    b = run(p).state()
    for x, y in zip(a, b):
        assert np.array_equal(x[perm], y)


def test_thread_count_does_not_change_bits():
    case = W.bumps_canal(nx=80, ny=20, lx=30.0, ly=10.0, x_dam=15.0,
                         steps=60)
    a = run(case, threads=1).state()
    b = run(case, threads=4).state()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ---------------------------------------------------------- mesh validation

def two_triangles():
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return xy, tri


def make(xy, tri, bnd=None, tag=None):
    n = tri.shape[0]
    return W.Case(name="t", xy=xy, tri=tri,
                  bnd=np.zeros((0, 2), np.int32) if bnd is None else bnd,
                  bnd_tag=np.zeros(0, np.int32) if tag is None else tag,
                  bc={}, z=np.zeros(n), manning=np.zeros(n), h=np.ones(n),
                  hu=np.zeros(n), hv=np.zeros(n))


def test_mesh_counts_and_orientation():
    xy, tri = two_triangles()
    tri[1] = tri[1][::-1]                       # clockwise input
    o = O.Oracle(make(xy, tri))
    assert o.counts() == dict(n_nodes=4, n_cells=2, n_edges=5, n_bnd_edges=4)
    area, inr, ccw = o.geometry()
    assert np.allclose(area, 0.5)
    assert np.allclose(inr, 2 * 0.5 / (2 + math.sqrt(2)))
    e = o.edges()
    inner = e["right"] >= 0
    assert inner.sum() == 1
    # normal of the diagonal points from the left to the right cell
    k = np.nonzero(inner)[0][0]
    cl = xy[ccw[e["left"][k]]].mean(0)
    cr = xy[ccw[e["right"][k]]].mean(0)
    assert np.dot(cr - cl, [e["nx"][k], e["ny"][k]]) > 0


@pytest.mark.parametrize("kind", ["degenerate", "range", "nonmanifold",
                                  "overlap", "segment", "dupseg", "tag"])
def test_mesh_errors(kind):
    xy, tri = two_triangles()
    bnd = tag = None
    if kind == "degenerate":                   # collinear nodes 0, 1, 4
        xy = np.vstack([xy, [2.0, 0.0]])
        tri = np.vstack([tri, [0, 1, 4]]).astype(np.int32)
    elif kind == "range":
        tri[0, 2] = 9
    elif kind == "nonmanifold":                # three cells on edge (0, 2)
        xy = np.vstack([xy, [2, 0.5]])
        tri = np.vstack([tri, [0, 2, 4]]).astype(np.int32)
    elif kind == "overlap":                    # both cells left of 0 -> 1
        xy = np.array([[0, 0], [1, 0], [1, 1], [0.2, 0.5]], float)
        tri = np.array([[0, 1, 2], [0, 1, 3]], np.int32)
    elif kind == "segment":
        bnd = np.array([[0, 2]], np.int32)     # the interior diagonal
        tag = np.array([1], np.int32)
    elif kind == "dupseg":
        bnd = np.array([[0, 1], [1, 0]], np.int32)
        tag = np.array([1, 2], np.int32)
    elif kind == "tag":
        bnd = np.array([[0, 1]], np.int32)
        tag = np.array([5000], np.int32)
    with pytest.raises(O.OracleError):
        O.Oracle(make(xy, tri, bnd, tag))


# ------------------------------------------------------- wall momentum balance

def test_wall_momentum_balance_under_impinging_flow():
    """Reading R11 (sec. 3.1): a wall edge passes only the hydrostatic
    pressure of its cell, g h^2 / 2 along the outward normal, whatever the
    velocity into the wall. On a flat, frictionless, closed basin the
    interior fluxes cancel in pairs and the bed adds nothing, so over one
    step the total momentum changes by exactly -dt * sum over wall edges of
    L (g/2) h_cell^2 n. The flow here runs obliquely into every wall; a
    mirror-state Riemann wall, a velocity-dependent wall flux or a wrong
    pressure factor breaks the balance at order one."""
    case = W.dam_break_canal(nx=60, ny=20, lx=60.0, ly=20.0)
    xy, tri = case.xy, case.tri.astype(np.int64)
    cen = xy[tri].mean(axis=1)
    n = tri.shape[0]
    case.h = 1.0 + 0.2 * np.sin(0.21 * cen[:, 0]) * np.cos(0.37 * cen[:, 1])
    case.hu = case.h * (0.8 + 0.3 * np.cos(0.17 * cen[:, 1]))
    case.hv = case.h * (-0.6 + 0.2 * np.sin(0.11 * cen[:, 0]))
    case.manning = np.zeros(n)
    case.z = np.zeros(n)
    o = O.Oracle(case)
    h0, hu0, hv0 = o.state()
    dt = 0.01
    o.run_dt(np.array([dt]))
    h1, hu1, hv1 = o.state()
    # areas (shoelace) and the wall edges with their cell, length and
    # outward normal, from the mesh alone
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    area = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) -
                        (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1]))
    owner = {}
    for t in range(n):
        for k in range(3):
            p, q = int(tri[t, k]), int(tri[t, (k + 1) % 3])
            owner.setdefault((min(p, q), max(p, q)), []).append(t)
    fx = fy = 0.0
    walls = 0
    for (p, q), cells in owner.items():
        if len(cells) != 1:
            continue
        t = cells[0]
        d = xy[q] - xy[p]
        L = math.hypot(d[0], d[1])
        nrm = np.array([d[1], -d[0]]) / L
        if np.dot(nrm, xy[p] - cen[t]) < 0.0:       # point away from the cell
            nrm = -nrm
        pres = L * 0.5 * G * h0[t] ** 2
        fx += pres * nrm[0]
        fy += pres * nrm[1]
        walls += 1
    assert walls == 2 * (60 + 20)
    # the flow impinges on the walls: momentum normal to them is not small
    assert np.max(np.abs(hu0)) > 0.5 and np.max(np.abs(hv0)) > 0.3
    dmx = math.fsum(area * (hu1 - hu0))
    dmy = math.fsum(area * (hv1 - hv0))
    assert abs(dmx - (-dt * fx)) <= 1e-11 * abs(dt * fx)
    assert abs(dmy - (-dt * fy)) <= 1e-11 * max(abs(dt * fy), 1e-3)
    # mass is untouched by the walls
    assert abs(math.fsum(area * (h1 - h0))) <= 1e-12 * math.fsum(area * h0)
