"""Seeded synthetic inputs for the explicit shallow-water finite-volume step.

This module builds meshes, bed and friction fields, boundary tags and initial
states. It holds none of the numerical method's arithmetic (no flux, no
source term, no update, no time step): only geometry needed to *place* data
(node coordinates, cell centroids, boundary-edge detection by topology).
Both the CPU oracle (through the tests) and the GPU library take their inputs
from here, so that the two sides see byte-identical arrays.

The workloads stand in for the paper's meshes (section 6), which are not
available:

* ``dam_break_canal``  -- a 1-D dam break in a flat, frictionless canal
  (the paper's section 6.3 test, scaled to 100 m x 20 m).
* ``bumps_canal``      -- the same canal refined to 1 000 x 500 squares, a dam
  break onto a dry bed over a seeded bed of Gaussian bumps, Manning n = 0.03.
* ``river``            -- a seeded meandering river reach standing in for the
  Mille Iles / Montreal river meshes of sections 6.4-6.5: jittered-point
  Delaunay mesh, thalweg + Perlin-noise bed, per-cell Manning n, an upstream
  inflow, a downstream fixed water level and a partly dry floodplain.

Boundary-condition kinds use the integer codes of the C interface
(``include/swe.h``): 0 wall, 1 transmissive, 2 inflow discharge,
3 fixed depth, 4 fixed water-surface elevation.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Tuple

import numpy as np

BC_WALL = 0
BC_TRANSMISSIVE = 1
BC_INFLOW = 2
BC_FIXED_DEPTH = 3
BC_FIXED_STAGE = 4

G_DEFAULT = 9.81
CFL_DEFAULT = 0.9
H_DRY_DEFAULT = 1e-6


@dataclasses.dataclass
class Case:
    """One complete input: mesh, fields, boundary conditions, initial state.

    Arrays use the caller's ("user") ordering. ``tri`` may list vertices in
    either orientation. ``bnd`` lists boundary segments as node pairs with a
    tag in ``bnd_tag``; unlisted boundary edges carry tag 0. ``bc`` maps a tag
    to ``(kind, value)``; tags absent from it are walls.
    """

    name: str
    xy: np.ndarray          # (n_nodes, 2) float64
    tri: np.ndarray         # (n_cells, 3) int32
    bnd: np.ndarray         # (n_bnd, 2) int32
    bnd_tag: np.ndarray     # (n_bnd,) int32
    bc: Dict[int, Tuple[int, float]]
    z: np.ndarray           # (n_cells,) bed elevation [m]
    manning: np.ndarray     # (n_cells,) Manning coefficient [s m^-1/3]
    h: np.ndarray           # (n_cells,) depth [m]
    hu: np.ndarray          # (n_cells,) discharge per width, x [m^2/s]
    hv: np.ndarray          # (n_cells,) discharge per width, y [m^2/s]
    g: float = G_DEFAULT
    cfl: float = CFL_DEFAULT
    h_dry: float = H_DRY_DEFAULT
    t_end: float = math.inf
    steps: int = 1
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    def centroids(self) -> np.ndarray:
        return self.xy[self.tri].mean(axis=1)

    def copy(self) -> "Case":
        return dataclasses.replace(
            self,
            xy=self.xy.copy(), tri=self.tri.copy(), bnd=self.bnd.copy(),
            bnd_tag=self.bnd_tag.copy(), bc=dict(self.bc), z=self.z.copy(),
            manning=self.manning.copy(), h=self.h.copy(), hu=self.hu.copy(),
            hv=self.hv.copy(), meta=dict(self.meta))


# --------------------------------------------------------------------------
# structured canal meshes
# --------------------------------------------------------------------------

def canal_mesh(nx: int, ny: int, lx: float, ly: float, x0: float = 0.0,
               y0: float = 0.0):
    """Rectangle [x0,x0+lx] x [y0,y0+ly] of nx x ny squares, each split along
    its south-west to north-east diagonal into two counter-clockwise triangles
    (the grid-point meshes of the paper's dam-break case, section 6.3).

    Returns ``xy, tri, bnd, bnd_tag`` with boundary tags 1 south, 2 east,
    3 north, 4 west.
    """
    xs = x0 + lx * np.arange(nx + 1, dtype=np.float64) / nx
    ys = y0 + ly * np.arange(ny + 1, dtype=np.float64) / ny
    X, Y = np.meshgrid(xs, ys)
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    a = (jj * (nx + 1) + ii).ravel()
    b = a + 1
    c = a + nx + 2
    d = a + nx + 1
    tri = np.empty((2 * a.size, 3), dtype=np.int32)
    tri[0::2] = np.stack([a, b, c], axis=1)
    tri[1::2] = np.stack([a, c, d], axis=1)
    i = np.arange(nx)
    j = np.arange(ny)
    south = np.stack([i, i + 1], axis=1)
    north = np.stack([ny * (nx + 1) + i + 1, ny * (nx + 1) + i], axis=1)
    east = np.stack([j * (nx + 1) + nx, (j + 1) * (nx + 1) + nx], axis=1)
    west = np.stack([(j + 1) * (nx + 1), j * (nx + 1)], axis=1)
    bnd = np.concatenate([south, east, north, west]).astype(np.int32)
    bnd_tag = np.concatenate([np.full(nx, 1), np.full(ny, 2), np.full(nx, 3),
                              np.full(ny, 4)]).astype(np.int32)
    return xy, tri, bnd, bnd_tag


def edge_list(case: "Case", seed: int = 0):
    """The case's mesh as an edge list: every pair of nodes that is a side of
    a triangle, once, with the one or two triangles on it and the boundary
    tag of a boundary edge (from ``bnd``/``bnd_tag``; 0 if unlisted and on
    interior edges). Topology only. Edges come in a seeded random order, and
    each edge's two node slots and two cell slots are swapped at random
    (independently), so a consumer cannot rely on any ordering.

    Returns ``edge_nodes (n, 2), edge_cells (n, 2) (-1 in one slot on the
    boundary), edge_tag (n,)``, all int32.
    """
    rng = np.random.default_rng(seed)
    tri = np.asarray(case.tri, dtype=np.int64)
    nc = tri.shape[0]
    p = tri.ravel()
    q = np.roll(tri, -1, axis=1).ravel()
    lo, hi = np.minimum(p, q), np.maximum(p, q)
    key = lo * (case.n_nodes + 1) + hi
    cell = np.repeat(np.arange(nc), 3)
    order = np.argsort(key, kind="stable")
    key, cell, lo, hi = key[order], cell[order], lo[order], hi[order]
    first = np.ones(key.size, bool)
    first[1:] = key[1:] != key[:-1]
    starts = np.flatnonzero(first)
    counts = np.diff(np.append(starts, key.size))
    if np.any(counts > 2):
        raise ValueError("a side is shared by more than two triangles")
    n = starts.size
    nodes = np.stack([lo[starts], hi[starts]], axis=1)
    cells = np.full((n, 2), -1, np.int64)
    cells[:, 0] = cell[starts]
    two = counts == 2
    cells[two, 1] = cell[starts[two] + 1]
    tags = np.zeros(n, np.int64)
    if len(case.bnd):
        b = np.asarray(case.bnd, dtype=np.int64)
        bkey = b.min(axis=1) * (case.n_nodes + 1) + b.max(axis=1)
        at = np.searchsorted(key[starts], bkey)
        tags[at] = case.bnd_tag
    perm = rng.permutation(n)
    nodes, cells, tags = nodes[perm], cells[perm], tags[perm]
    swap_n = rng.random(n) < 0.5
    nodes[swap_n] = nodes[swap_n][:, ::-1]
    swap_c = rng.random(n) < 0.5
    cells[swap_c] = cells[swap_c][:, ::-1]
    return (nodes.astype(np.int32), cells.astype(np.int32),
            tags.astype(np.int32))


def _zeros(n):
    return np.zeros(n, dtype=np.float64)


def dam_break_canal(nx: int = 100, ny: int = 20, lx: float = 100.0,
                    ly: float = 20.0, h_left: float = 1.0,
                    h_right: float = 0.5, x_dam: float = 50.0,
                    t_end: float = 5.0) -> Case:
    """Flat frictionless canal, walls all round, dam at x = x_dam, still water
    (h_left upstream, h_right downstream). Default: 100 x 20 squares of 1 m,
    4 000 triangles, run to t = 5 s (compared with Stoker's solution)."""
    xy, tri, bnd, tag = canal_mesh(nx, ny, lx, ly)
    n = tri.shape[0]
    cx = xy[tri].mean(axis=1)[:, 0]
    h = np.where(cx < x_dam, h_left, h_right).astype(np.float64)
    return Case(name=f"dam-break-canal-{nx}x{ny}", xy=xy, tri=tri, bnd=bnd,
                bnd_tag=tag, bc={}, z=_zeros(n), manning=_zeros(n), h=h,
                hu=_zeros(n), hv=_zeros(n), t_end=t_end, steps=10**9,
                meta=dict(h_left=h_left, h_right=h_right, x_dam=x_dam,
                          lx=lx, ly=ly))


def gaussian_bumps(points: np.ndarray, lx: float, ly: float, seed: int,
                   n_bumps: int = 20, z_max: float = 0.2) -> np.ndarray:
    """Sum of ``n_bumps`` seeded Gaussians on [0,lx] x [0,ly], centres
    uniform, widths sigma ~ U[1,4] m, amplitudes ~ U[0.05,0.2] m, rescaled so
    that the maximum over ``points`` does not exceed ``z_max``."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    cxy = rng.uniform([0.0, 0.0], [lx, ly], size=(n_bumps, 2))
    sig = rng.uniform(1.0, 4.0, size=n_bumps)
    amp = rng.uniform(0.05, 0.2, size=n_bumps)
    z = np.zeros(points.shape[0])
    for k in range(n_bumps):
        d2 = ((points - cxy[k]) ** 2).sum(axis=1)
        z += amp[k] * np.exp(-d2 / (2.0 * sig[k] ** 2))
    zm = z.max() if z.size else 0.0
    if zm > z_max:
        z *= z_max / zm
    return z


def bumps_canal(nx: int = 1000, ny: int = 500, lx: float = 100.0,
                ly: float = 20.0, seed: int = 2, manning: float = 0.03,
                h_left: float = 1.0, x_dam: float = 50.0,
                steps: int = 2000) -> Case:
    """Dam break onto a dry bed over seeded Gaussian bumps: depth h_left for
    x < x_dam, dry beyond, Manning n uniform, walls all round (closed)."""
    xy, tri, bnd, tag = canal_mesh(nx, ny, lx, ly)
    n = tri.shape[0]
    cen = xy[tri].mean(axis=1)
    z = gaussian_bumps(cen, lx, ly, seed)
    h = np.where(cen[:, 0] < x_dam, h_left, 0.0).astype(np.float64)
    return Case(name=f"bumps-canal-{nx}x{ny}", xy=xy, tri=tri, bnd=bnd,
                bnd_tag=tag, bc={}, z=z, manning=np.full(n, manning), h=h,
                hu=_zeros(n), hv=_zeros(n), steps=steps,
                meta=dict(seed=seed, lx=lx, ly=ly))


def wet_canal(nx: int = 3600, ny: int = 1806, manning: float = 0.03,
              h_left: float = 2.0, h_right: float = 1.0,
              u0: float = 0.5) -> Case:
    """Every cell wet and moving: squares of 1 m, flat bed, Manning n
    uniform, depth h_left upstream of the middle and h_right downstream, all
    with velocity u0 along the canal, walls all round. The step's uniform
    case: every edge a wet-wet flux, every cell a Manning update (13 M cells
    by default)."""
    xy, tri, bnd, tag = canal_mesh(nx, ny, float(nx), float(ny))
    n = tri.shape[0]
    cx = xy[tri].mean(axis=1)[:, 0]
    h = np.where(cx < nx / 2.0, h_left, h_right).astype(np.float64)
    return Case(name=f"wet-canal-{nx}x{ny}", xy=xy, tri=tri, bnd=bnd,
                bnd_tag=tag, bc={}, z=_zeros(n), manning=np.full(n, manning),
                h=h, hu=u0 * h, hv=_zeros(n), steps=1000,
                meta=dict(lx=float(nx), ly=float(ny)))


def lake_at_rest(nx: int = 100, ny: int = 40, lx: float = 100.0,
                 ly: float = 20.0, seed: int = 2, eta: float = 0.12,
                 manning: float = 0.03, steps: int = 2000) -> Case:
    """Still water at surface elevation ``eta`` over the seeded bumps; the
    bump tops above ``eta`` are dry."""
    xy, tri, bnd, tag = canal_mesh(nx, ny, lx, ly)
    n = tri.shape[0]
    cen = xy[tri].mean(axis=1)
    z = gaussian_bumps(cen, lx, ly, seed)
    h = np.maximum(0.0, eta - z)
    return Case(name=f"lake-at-rest-{nx}x{ny}", xy=xy, tri=tri, bnd=bnd,
                bnd_tag=tag, bc={}, z=z, manning=np.full(n, manning), h=h,
                hu=_zeros(n), hv=_zeros(n), steps=steps,
                meta=dict(seed=seed, eta=eta))


# --------------------------------------------------------------------------
# Perlin gradient noise (Perlin 1985; quintic fade of Perlin 2002)
# --------------------------------------------------------------------------

def perlin2(x: np.ndarray, y: np.ndarray, rng: np.random.Generator,
            period: int = 4096) -> np.ndarray:
    """2-D gradient noise: unit gradients on the integer lattice (drawn from
    ``rng`` through a permutation table, as in Perlin's method), dot products
    with the offsets to the four surrounding lattice corners, blended with the
    quintic fade 6t^5 - 15t^4 + 10t^3."""
    perm = rng.permutation(period)
    ang = rng.uniform(0.0, 2.0 * np.pi, size=period)
    gx, gy = np.cos(ang), np.sin(ang)
    xi = np.floor(x).astype(np.int64)
    yi = np.floor(y).astype(np.int64)
    fx = x - xi
    fy = y - yi

    def grad(ix, iy, dx, dy):
        k = perm[(perm[ix % period] + iy) % period]
        return gx[k] * dx + gy[k] * dy

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    n00 = grad(xi, yi, fx, fy)
    n10 = grad(xi + 1, yi, fx - 1.0, fy)
    n01 = grad(xi, yi + 1, fx, fy - 1.0)
    n11 = grad(xi + 1, yi + 1, fx - 1.0, fy - 1.0)
    u = fade(fx)
    v = fade(fy)
    nx0 = n00 + u * (n10 - n00)
    nx1 = n01 + u * (n11 - n01)
    return nx0 + v * (nx1 - nx0)


def perlin_octaves(x, y, rng, base_wavelength=200.0, octaves=3):
    out = np.zeros_like(x)
    for k in range(octaves):
        lam = base_wavelength / 2 ** k
        out += 0.5 ** k * perlin2(x / lam, y / lam, rng)
    return out


# --------------------------------------------------------------------------
# meandering river reach
# --------------------------------------------------------------------------

RIVER_LENGTH = 12_000.0
RIVER_HALF_WIDTH = 550.0
RIVER_CHANNEL_HALF_WIDTH = 75.0


def _strip_points(x0, x1, hw, s, rng, lattice):
    """Points of one strip [x0,x1] x [-hw,hw] of the along-channel parameter
    plane: equally spaced points on the four sides plus the jittered
    triangular-lattice points that lie at least s/2 inside."""
    nv = max(1, int(round(2 * hw / s)))
    yv = -hw + 2 * hw * np.arange(nv + 1) / nv
    nh = max(1, int(round((x1 - x0) / s)))
    xh = x0 + (x1 - x0) * np.arange(1, nh) / nh
    side = np.concatenate([
        np.stack([np.full(nv + 1, x0), yv], 1),
        np.stack([np.full(nv + 1, x1), yv], 1),
        np.stack([xh, np.full(xh.size, -hw)], 1),
        np.stack([xh, np.full(xh.size, hw)], 1)])
    lx, ly = lattice
    m = (lx > x0 + 0.5 * s) & (lx < x1 - 0.5 * s)
    px = lx[m] + rng.uniform(-0.25 * s, 0.25 * s, m.sum())
    py = ly[m] + rng.uniform(-0.25 * s, 0.25 * s, m.sum())
    inner = np.stack([px, py], 1)
    return side, inner


def _triangulate_strip(args):
    from scipy.spatial import Delaunay
    pts = args
    d = Delaunay(pts)
    return d.simplices.astype(np.int32)


def river(n_target: int = 13_000_000, seed: int = 3, n_strips: int = 16,
          inflow_q: float = 500.0, stage_offset: float = 5.3,
          steps: int = 1000, shuffle: bool = True, workers: int = 8,
          length: float = RIVER_LENGTH,
          half_width: float = RIVER_HALF_WIDTH) -> Case:
    """Seeded meandering river reach of about ``n_target`` triangles.

    The mesh is a Delaunay triangulation of jittered triangular-lattice
    points in the along-channel parameter plane (xi, eta) in
    [0, length] x [-half_width, half_width], triangulated in ``n_strips``
    strips that share their separating lines of points, then mapped to the
    physical plane by x = xi, y = eta + yc(xi) with the centreline
    yc(x) = 300 sin(2 pi x/3000 + p1) + 80 sin(2 pi x/1100 + p2).

    Bed: thalweg zt = 10 - 2e-4 x; channel (|d| <= 75 m) zt + 5 (d/75)^2;
    floodplain zt + 5 + min(1, (|d|-75)/300); plus three octaves of Perlin
    noise (base wavelength 200 m) scaled to a standard deviation of 0.5 m.
    Manning n per cell ~ U[0.02, 0.05]. Boundary: the channel section of the
    upstream end (x = 0, |d| <= 75) is an inflow of ``inflow_q`` m^3/s
    (tag 1); the channel section of the downstream end is held at the
    initial water level (tag 2); everything else is a wall. Initial state: an
    inclined water plane eta = zt + stage_offset at rest (the inclined-plane
    start of the paper's section 6.5), dry where it lies below the bed.
    Cells are shuffled (seeded) so that locality has to be recovered.
    """
    ss = np.random.SeedSequence(seed).spawn(6)
    r_phase = np.random.default_rng(ss[0])
    r_jit = np.random.default_rng(ss[1])
    r_noise = np.random.default_rng(ss[2])
    r_mann = np.random.default_rng(ss[3])
    r_shuf = np.random.default_rng(ss[4])
    p1, p2 = r_phase.uniform(0.0, 2 * np.pi, 2)

    area = length * 2 * half_width
    s = math.sqrt(area * 4.0 / (math.sqrt(3.0) * n_target))
    dy = s * math.sqrt(3.0) / 2.0
    nrow = int(math.floor((2 * half_width - s) / dy)) + 1
    rows = -half_width + 0.5 * s + dy * np.arange(nrow)
    rows = rows[rows <= half_width - 0.5 * s]
    ncol = int(math.floor(length / s)) + 2
    lat_x = (np.arange(ncol)[None, :] * s
             + 0.5 * s * (np.arange(rows.size)[:, None] % 2)).ravel()
    lat_y = np.repeat(rows, ncol)

    edges_x = np.linspace(0.0, length, n_strips + 1)
    # snap strip separators to the side-point spacing so neighbours share them
    nh_tot = int(round(length / s))
    edges_x = np.round(edges_x / length * nh_tot) / nh_tot * length
    strips = []
    for k in range(n_strips):
        m = (lat_x > edges_x[k] - s) & (lat_x < edges_x[k + 1] + s)
        side, inner = _strip_points(edges_x[k], edges_x[k + 1], half_width, s,
                                    r_jit, (lat_x[m], lat_y[m]))
        strips.append((side, inner))

    if workers > 1:
        # threads, not processes: Qhull releases the GIL, and no process is
        # forked (a forked child of a profiled or GPU-initialised process can
        # hang on exit)
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(min(workers, n_strips)) as ex:
            simp = list(ex.map(_triangulate_strip,
                               [np.concatenate(st) for st in strips]))
    else:
        simp = [_triangulate_strip(np.concatenate(st)) for st in strips]

    # global node numbering: side points are deduplicated by exact coordinates
    all_pts = []
    all_tri = []
    key_to_id: Dict[Tuple[float, float], int] = {}
    n_nodes = 0
    for (side, inner), tri in zip(strips, simp):
        ids = np.empty(side.shape[0] + inner.shape[0], dtype=np.int64)
        for q in range(side.shape[0]):
            kk = (float(side[q, 0]), float(side[q, 1]))
            j = key_to_id.get(kk)
            if j is None:
                j = n_nodes
                key_to_id[kk] = j
                all_pts.append(side[q:q + 1])
                n_nodes += 1
            ids[q] = j
        ids[side.shape[0]:] = n_nodes + np.arange(inner.shape[0])
        all_pts.append(inner)
        n_nodes += inner.shape[0]
        all_tri.append(ids[tri])
    P = np.concatenate(all_pts)
    T = np.concatenate(all_tri)
    # drop degenerate (zero-area) triangles Qhull may leave on straight sides
    a2 = ((P[T[:, 1], 0] - P[T[:, 0], 0]) * (P[T[:, 2], 1] - P[T[:, 0], 1])
          - (P[T[:, 2], 0] - P[T[:, 0], 0]) * (P[T[:, 1], 1] - P[T[:, 0], 1]))
    T = T[np.abs(a2) > 1e-9 * s * s]

    def yc(x):
        return (300.0 * np.sin(2 * np.pi * x / 3000.0 + p1)
                + 80.0 * np.sin(2 * np.pi * x / 1100.0 + p2))

    xy = np.stack([P[:, 0], P[:, 1] + yc(P[:, 0])], axis=1)
    tri = T.astype(np.int32)
    n = tri.shape[0]

    cen_p = P[T].mean(axis=1)          # centroid in the parameter plane
    d = np.abs(cen_p[:, 1])
    xc = cen_p[:, 0]
    zt = 10.0 - 2e-4 * xc
    z = np.where(d <= RIVER_CHANNEL_HALF_WIDTH,
                 zt + 5.0 * (d / RIVER_CHANNEL_HALF_WIDTH) ** 2,
                 zt + 5.0 + np.minimum(1.0, (d - RIVER_CHANNEL_HALF_WIDTH)
                                       / 300.0))
    cen = xy[tri].mean(axis=1)
    noise = perlin_octaves(cen[:, 0], cen[:, 1], r_noise)
    noise *= 0.5 / noise.std()
    z = z + noise
    manning = r_mann.uniform(0.02, 0.05, n)
    eta = zt + stage_offset
    h = np.maximum(0.0, eta - z)

    # boundary edges: half-edges that occur once
    he = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    key = np.minimum(he[:, 0], he[:, 1]).astype(np.int64) * n_nodes + \
        np.maximum(he[:, 0], he[:, 1])
    uk, cnt = np.unique(key, return_counts=True)
    bkey = uk[cnt == 1]
    b0 = (bkey // n_nodes).astype(np.int32)
    b1 = (bkey % n_nodes).astype(np.int32)
    mid = 0.5 * (P[b0] + P[b1])
    tol = 1e-6 * s
    chan = np.abs(mid[:, 1]) <= RIVER_CHANNEL_HALF_WIDTH
    up = (np.abs(P[b0, 0]) < tol) & (np.abs(P[b1, 0]) < tol) & chan
    down = (np.abs(P[b0, 0] - length) < tol) & \
        (np.abs(P[b1, 0] - length) < tol) & chan
    sel = up | down
    bnd = np.stack([b0[sel], b1[sel]], 1).astype(np.int32)
    bnd_tag = np.where(up[sel], 1, 2).astype(np.int32)
    stage_out = 10.0 - 2e-4 * length + stage_offset
    bc = {1: (BC_INFLOW, float(inflow_q)), 2: (BC_FIXED_STAGE, stage_out)}

    if shuffle:
        perm = r_shuf.permutation(n)
        tri, z, manning, h = tri[perm], z[perm], manning[perm], h[perm]
    return Case(name=f"river-{n}", xy=xy, tri=np.ascontiguousarray(tri),
                bnd=bnd, bnd_tag=bnd_tag, bc=bc, z=z, manning=manning, h=h,
                hu=_zeros(n), hv=_zeros(n), steps=steps,
                meta=dict(seed=seed, spacing=s, phases=(p1, p2),
                          n_strips=n_strips, inflow_q=inflow_q,
                          stage_out=stage_out))


# --------------------------------------------------------------------------
# the three standard workloads
# --------------------------------------------------------------------------

def ensemble_members(n_members: int = 256, seed: int = 4,
                     min_cells: int = 10_000, max_cells: int = 200_000,
                     steps: int = 500, workers: int = 8) -> list:
    """Uncertainty ensemble of river runs (the sampled inflow and friction of
    sec. 6.4.3): member sizes ~ U[min_cells, max_cells] triangles, one
    Manning coefficient n ~ U[0.02, 0.05] and one inflow Q ~ U[200, 800]
    m^3/s per member, all on the reach and bed of the same seeded generator
    (seed ``seed``) meshed at their own resolution. The draws come from
    numpy SeedSequence(seed) in the order sizes, n, Q. Members are built in
    ``workers`` threads."""
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    sizes = rng.integers(min_cells, max_cells + 1, n_members)
    mann = rng.uniform(0.02, 0.05, n_members)
    flow = rng.uniform(200.0, 800.0, n_members)

    def one(k):
        c = river(n_target=int(sizes[k]), seed=seed, inflow_q=float(flow[k]),
                  steps=steps, workers=1)
        c.manning = np.full(c.n_cells, float(mann[k]))
        c.name = f"ensemble-member-{k}"
        return c

    if workers > 1:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(one, range(n_members)))
    return [one(k) for k in range(n_members)]


def config(k: int, **kw):
    """Standard workloads: 1 dam-break canal (4 000 cells, to t = 5 s),
    2 bumps canal (1 000 000 cells, 2 000 steps), 3 river (about 13 M cells,
    1 000 steps), 4 ensemble of 256 river runs (about 27 M cells in all, 500
    steps each; a list of cases)."""
    if k == 1:
        return dam_break_canal(**kw)
    if k == 2:
        return bumps_canal(**kw)
    if k == 3:
        return river(**kw)
    if k == 4:
        return ensemble_members(**kw)
    raise ValueError(f"unknown workload {k}")
