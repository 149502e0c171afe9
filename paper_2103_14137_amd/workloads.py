"""Seeded synthetic scenes, lamp poses and lamp models.

This module only *produces inputs*: triangle meshes (float32 vertices, int32
indices), candidate lamp base positions and lamp models.  It contains none of
the method's arithmetic (no surface elements, no irradiance, no visibility),
so both the HIP path and the CPU oracle can consume its output without sharing
any computation.

Conventions shared by every generator
-------------------------------------
* Units are metres and watts.  The floor is the plane z = 0.
* Every triangle is wound so that its right-hand normal (v1 - v0) x (v2 - v0)
  points into free space: room shells are wound inward, obstacles outward.
  This is the orientation the paper's visibility condition needs for the
  surface normal (Sec. IV-C, the inverse-square law and the strict
  front-facing condition that follows it).
* Every closed box is generated on a lattice whose vertices are shared by the
  faces that meet at them, so each box is a watertight, consistently oriented
  triangle mesh.
* A pose is a lamp base position (x, y) on the floor.  A lamp is a list of
  point sources at heights dz above the base, each with its own power; the
  paper approximates an extended lamp by evenly distributed point sources of
  equal power (Sec. IV-C, "Non-Point Light Sources").

Workloads (sizes follow the configurations the hot path is measured on):
  box_room   4 x 4 x 3 m room, 0.5 m cube, 200 poses, 80 W point lamp
  ward       8 x 6 x 3 m ward, 6 beds + 10 cuboids, ~52k triangles,
             5,000 poses, 8-source tower lamp (8 x 20 W)
  floorplan  12 rooms with doorways, ~500k triangles, 20,000 poses, tower lamp
  batch      64 rooms of uneven size (2k-80k triangles, 500-8,000 poses)
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclass
class Mesh:
    verts: np.ndarray  # float32 [V, 3]
    tris: np.ndarray   # int32 [N, 3]

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])


@dataclass
class Lamp:
    dz: np.ndarray     # float32 [S] source heights above the pose base point
    power: np.ndarray  # float32 [S] radiant flux of each source in W

    @property
    def n_src(self) -> int:
        return int(self.dz.shape[0])


@dataclass
class Workload:
    name: str
    mesh: Mesh
    poses: np.ndarray  # float32 [K, 2] lamp base positions
    lamp: Lamp
    meta: dict = field(default_factory=dict)
    free_fn: object = None   # (X, Y) -> bool array: where the lamp base may stand
    bounds: tuple = None     # ((x0, x1), (y0, y1)) of the pose region

    @property
    def K(self) -> int:
        return int(self.poses.shape[0])

    @property
    def N(self) -> int:
        return self.mesh.n_tris


def point_lamp(height: float = 1.0, power: float = 80.0) -> Lamp:
    """Isotropic point lamp 1 m above the base, 80 W (Sec. V: P = 80 W; the
    2.5D experiment holds the light at 1 m)."""
    return Lamp(np.array([height], np.float32), np.array([power], np.float32))


def tower_lamp(n: int = 8, spacing: float = 0.2, power_each: float = 20.0) -> Lamp:
    """Tower lamp as n stacked point sources at spacing, 2*spacing, ...,
    n*spacing above the base, power_each W apiece."""
    dz = np.array([spacing * (j + 1) for j in range(n)], np.float32)
    return Lamp(dz, np.full(n, power_each, np.float32))


# ----------------------------------------------------------------------------
# mesh construction
# ----------------------------------------------------------------------------
def _subdiv(a: float, b: float, n: int) -> np.ndarray:
    """n equal cells on [a, b], endpoints exact."""
    k = np.arange(n + 1, dtype=np.float64)
    pts = a + (b - a) * k / n
    pts[0], pts[-1] = a, b
    return pts


def _ncells(length: float, h: float) -> int:
    return max(1, int(math.ceil(length / h - 1e-9)))


class MeshBuilder:
    """Accumulates float64 vertex blocks and int triangle blocks."""

    def __init__(self):
        self._v = []
        self._t = []
        self._nv = 0

    def add(self, verts: np.ndarray, tris: np.ndarray) -> None:
        self._v.append(np.asarray(verts, np.float64))
        self._t.append(np.asarray(tris, np.int64) + self._nv)
        self._nv += len(verts)

    def mesh(self) -> Mesh:
        v = np.concatenate(self._v).astype(np.float32)
        t = np.concatenate(self._t).astype(np.int32)
        return Mesh(np.ascontiguousarray(v), np.ascontiguousarray(t))


def _quad_tris(p00, p10, p11, p01, flip):
    """Two triangles of the quad p00-p10-p11-p01 (arrays of vertex ids).  With
    flip False their right-hand normal is (p10-p00) x (p01-p00)."""
    if not flip:
        return np.stack([np.stack([p00, p10, p11], -1), np.stack([p00, p11, p01], -1)], 1).reshape(-1, 3)
    return np.stack([np.stack([p00, p11, p10], -1), np.stack([p00, p01, p11], -1)], 1).reshape(-1, 3)


def box_surface(lo, hi, counts, inward: bool, yaw: float = 0.0):
    """Closed lattice surface of the box [lo, hi] with counts[a] cells along
    axis a.  Outward winding unless inward.  yaw rotates the box about the
    vertical axis through its centre.  Returns float64 verts, int tris."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    n = [int(c) for c in counts]
    axes = [_subdiv(lo[a], hi[a], n[a]) for a in range(3)]
    vid = -np.ones((n[0] + 1, n[1] + 1, n[2] + 1), np.int64)
    on = np.zeros_like(vid, dtype=bool)
    on[[0, -1], :, :] = True
    on[:, [0, -1], :] = True
    on[:, :, [0, -1]] = True
    idx = np.argwhere(on)
    vid[tuple(idx.T)] = np.arange(len(idx))
    verts = np.stack([axes[0][idx[:, 0]], axes[1][idx[:, 1]], axes[2][idx[:, 2]]], -1)
    tris = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3  # cyclic, so e_b x e_c = e_a
        for side, sgn in ((0, -1), (n[a], +1)):
            want = -sgn if inward else sgn
            u, v = np.meshgrid(np.arange(n[b]), np.arange(n[c]), indexing="ij")
            u, v = u.ravel(), v.ravel()

            def P(du, dv):
                ijk = [None, None, None]
                ijk[a] = np.full_like(u, side)
                ijk[b] = u + du
                ijk[c] = v + dv
                return vid[ijk[0], ijk[1], ijk[2]]

            tris.append(_quad_tris(P(0, 0), P(1, 0), P(1, 1), P(0, 1), flip=(want < 0)))
    tris = np.concatenate(tris)
    if yaw != 0.0:
        cx, cy = 0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1])
        cs, sn = math.cos(yaw), math.sin(yaw)
        x, y = verts[:, 0] - cx, verts[:, 1] - cy
        verts = verts.copy()
        verts[:, 0] = cx + cs * x - sn * y
        verts[:, 1] = cy + sn * x + cs * y
    return verts, tris


def box_tri_count(dims, h) -> int:
    nx, ny, nz = (_ncells(d, h) for d in dims)
    return 4 * (nx * ny + ny * nz + nx * nz)


class FaceSet:
    """Axis-aligned gridded rectangles with optional rectangular holes, merged
    into one mesh with exact-coordinate vertex sharing (used for rooms joined
    by doorway tunnels)."""

    def __init__(self):
        self._key = {}
        self._verts = []
        self._tris = []

    def _vid(self, p):
        k = (float(p[0]), float(p[1]), float(p[2]))
        i = self._key.get(k)
        if i is None:
            i = len(self._verts)
            self._key[k] = i
            self._verts.append(k)
        return i

    def rect(self, axis, coord, ubreaks, vbreaks, h, normal_sign, holes=()):
        """Rectangle in the plane x_axis = coord.  ubreaks / vbreaks are sorted
        break coordinates along the two in-plane axes (b, c) = (axis+1, axis+2)
        mod 3; every interval between breaks is subdivided into cells of size
        <= h.  Cells whose centre lies inside a hole (u0, u1, v0, v1) are
        skipped.  normal_sign is the sign of the normal along axis."""
        us = np.concatenate([_subdiv(ubreaks[i], ubreaks[i + 1], _ncells(ubreaks[i + 1] - ubreaks[i], h))[:-1]
                             for i in range(len(ubreaks) - 1)] + [np.array([ubreaks[-1]])])
        vs = np.concatenate([_subdiv(vbreaks[i], vbreaks[i + 1], _ncells(vbreaks[i + 1] - vbreaks[i], h))[:-1]
                             for i in range(len(vbreaks) - 1)] + [np.array([vbreaks[-1]])])
        b, c = (axis + 1) % 3, (axis + 2) % 3
        ids = np.empty((len(us), len(vs)), np.int64)
        for i, uu in enumerate(us):
            for j, vv in enumerate(vs):
                p = [0.0, 0.0, 0.0]
                p[axis], p[b], p[c] = coord, uu, vv
                ids[i, j] = self._vid(p)
        uc = 0.5 * (us[:-1] + us[1:])
        vc = 0.5 * (vs[:-1] + vs[1:])
        keep = np.ones((len(uc), len(vc)), bool)
        for (u0, u1, v0, v1) in holes:
            keep &= ~(((uc > u0) & (uc < u1))[:, None] & ((vc > v0) & (vc < v1))[None, :])
        iu, jv = np.nonzero(keep)
        t = _quad_tris(ids[iu, jv], ids[iu + 1, jv], ids[iu + 1, jv + 1], ids[iu, jv + 1], flip=(normal_sign < 0))
        self._tris.append(t)

    def add_mesh(self, verts, tris):
        base = len(self._verts)
        for p in verts:
            self._verts.append((float(p[0]), float(p[1]), float(p[2])))
        self._tris.append(np.asarray(tris, np.int64) + base)

    def mesh(self) -> Mesh:
        v = np.asarray(self._verts, np.float64).astype(np.float32)
        t = np.concatenate(self._tris).astype(np.int32)
        return Mesh(np.ascontiguousarray(v), np.ascontiguousarray(t))


# ----------------------------------------------------------------------------
# obstacles and free-space pose grids
# ----------------------------------------------------------------------------
@dataclass
class Footprint:
    cx: float
    cy: float
    w: float    # extent along the local x axis
    d: float    # extent along the local y axis
    yaw: float


def _dist_to_footprints(px, py, fps):
    """Distance from points to the nearest rotated-rectangle footprint."""
    best = np.full(px.shape, np.inf)
    for f in fps:
        cs, sn = math.cos(f.yaw), math.sin(f.yaw)
        x, y = px - f.cx, py - f.cy
        lx = cs * x + sn * y
        ly = -sn * x + cs * y
        dx = np.maximum(np.abs(lx) - 0.5 * f.w, 0.0)
        dy = np.maximum(np.abs(ly) - 0.5 * f.d, 0.0)
        best = np.minimum(best, np.hypot(dx, dy))
    return best


def _largest_component(free: np.ndarray) -> np.ndarray:
    """Mask of the largest 4-connected component of a boolean grid."""
    lab = -np.ones(free.shape, np.int64)
    sizes = []
    nx, ny = free.shape
    for i0, j0 in zip(*np.nonzero(free)):
        if lab[i0, j0] >= 0:
            continue
        cid = len(sizes)
        stack = [(i0, j0)]
        lab[i0, j0] = cid
        n = 0
        while stack:
            i, j = stack.pop()
            n += 1
            for a, b in ((i + 1, j), (i - 1, j), (i, j + 1), (i, j - 1)):
                if 0 <= a < nx and 0 <= b < ny and free[a, b] and lab[a, b] < 0:
                    lab[a, b] = cid
                    stack.append((a, b))
        sizes.append(n)
    if not sizes:
        return np.zeros_like(free)
    return lab == int(np.argmax(sizes))


def free_grid(free_fn, bounds, h):
    """Grid points (x0 + i h, y0 + j h) inside bounds where free_fn is True,
    restricted to the largest 4-connected component."""
    (x0, x1), (y0, y1) = bounds
    xs = x0 + h * np.arange(int(math.floor((x1 - x0) / h)) + 1)
    ys = y0 + h * np.arange(int(math.floor((y1 - y0) / h)) + 1)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    free = free_fn(X, Y)
    comp = _largest_component(free)
    return np.stack([X[comp], Y[comp]], -1)


def occupancy(w: "Workload", cell: float = 0.05):
    """Free-space grid for the route stage: cells of side `cell` over the
    pose region grown by one cell; a cell is free when its centre lies
    within one half-diagonal of free space (free_fn with the clearance
    reduced by cell / sqrt(2)), so that every pose's cell is free.  Returns
    (free uint8 [H, W] with row = y index, column = x index, x0, y0): cell
    (r, c) covers [x0 + c cell, x0 + (c + 1) cell) x [y0 + r cell, ...)."""
    if w.free_fn is None:
        raise ValueError(f"{w.name}: no free-space description")
    (bx0, bx1), (by0, by1) = w.bounds
    x0, y0 = bx0 - cell, by0 - cell
    W = int(math.ceil((bx1 + cell - x0) / cell))
    H = int(math.ceil((by1 + cell - y0) / cell))
    cx = x0 + cell * (np.arange(W) + 0.5)
    cy = y0 + cell * (np.arange(H) + 0.5)
    X, Y = np.meshgrid(cx, cy, indexing="xy")
    free = w.free_fn(X, Y, slack=cell / math.sqrt(2.0))
    return free.astype(np.uint8), np.float32(x0), np.float32(y0)


def pose_grid(free_fn, bounds, K, rng, h0=0.25, shrink=0.8):
    """K poses: the free grid at spacing h0, refined geometrically until its
    largest component holds at least K points, then a seeded subsample of K
    points kept in grid order."""
    h = h0
    while True:
        pts = free_grid(free_fn, bounds, h)
        if len(pts) >= K:
            break
        h *= shrink
    sel = np.sort(rng.choice(len(pts), size=K, replace=False))
    return pts[sel].astype(np.float32), h


def _place_cuboid(rng, room_lo, room_hi, dims, margin=0.02):
    """Uniform centre (footprint kept inside the room) and uniform yaw."""
    w, d, _ = dims
    yaw = float(rng.uniform(0.0, 2.0 * math.pi))
    cs, sn = abs(math.cos(yaw)), abs(math.sin(yaw))
    hx = 0.5 * (cs * w + sn * d) + margin
    hy = 0.5 * (sn * w + cs * d) + margin
    cx = float(rng.uniform(room_lo[0] + hx, room_hi[0] - hx))
    cy = float(rng.uniform(room_lo[1] + hy, room_hi[1] - hy))
    return Footprint(cx, cy, w, d, yaw)


def _cuboid_mesh(fp: Footprint, height: float, h: float):
    lo = (fp.cx - 0.5 * fp.w, fp.cy - 0.5 * fp.d, 0.0)
    hi = (fp.cx + 0.5 * fp.w, fp.cy + 0.5 * fp.d, height)
    counts = (_ncells(fp.w, h), _ncells(fp.d, h), _ncells(height, h))
    return box_surface(lo, hi, counts, inward=False, yaw=fp.yaw)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------
def box_room(seed: int = 0, cell: float = 0.4, K: int = 200) -> Workload:
    """4 x 4 x 3 m room gridded at L / ceil(L / cell) per axis (walls, floor
    and ceiling: 1,040 triangles at cell = 0.4), plus one axis-aligned 0.5 m
    cube standing on the floor with its lower corner at a seeded position in
    [0.75, 2.75]^2 (12 triangles).  Poses: 0.25 m grid, at least 0.10 m from
    the cube footprint, seeded subsample of K.  Point lamp, 80 W, 1 m high."""
    rng = np.random.default_rng(seed)
    L = (4.0, 4.0, 3.0)
    mb = MeshBuilder()
    mb.add(*box_surface((0, 0, 0), L, [_ncells(l, cell) for l in L], inward=True))
    x0, y0 = (float(v) for v in rng.uniform(0.75, 2.75, size=2))
    s = 0.5
    mb.add(*box_surface((x0, y0, 0.0), (x0 + s, y0 + s, s), (1, 1, 1), inward=False))
    fp = [Footprint(x0 + 0.5 * s, y0 + 0.5 * s, s, s, 0.0)]

    def free_fn(X, Y, slack=0.0):
        return _dist_to_footprints(X, Y, fp) > 0.10 - slack

    bounds = ((0.25, 3.75), (0.25, 3.75))
    poses, h = pose_grid(free_fn, bounds, K, rng, h0=0.25)
    return Workload("box_room", mb.mesh(), poses, point_lamp(),
                    dict(seed=seed, cube_lo=(x0, y0, 0.0), cube_size=s, room=L, pose_spacing=h), free_fn, bounds)


def _room_with_cuboids(rng, L, beds, n_cuboids, cell, clearance, K, h0=0.25):
    """Room shell (inward) of size L with `beds` 2 x 1 x 0.6 m cuboids and
    n_cuboids cuboids with edges ~ U[0.3, 1.2] m, all standing on the floor
    with uniform centre and yaw.  Poses: free grid with `clearance` from the
    walls and from every footprint."""
    mb = MeshBuilder()
    mb.add(*box_surface((0, 0, 0), L, [_ncells(l, cell) for l in L], inward=True))
    fps, heights = [], []
    for _ in range(beds):
        fp = _place_cuboid(rng, (0, 0), L[:2], (2.0, 1.0, 0.6))
        fps.append(fp)
        heights.append(0.6)
    for _ in range(n_cuboids):
        dims = tuple(float(v) for v in rng.uniform(0.3, 1.2, size=3))
        fp = _place_cuboid(rng, (0, 0), L[:2], dims)
        fps.append(fp)
        heights.append(dims[2])
    for fp, ht in zip(fps, heights):
        mb.add(*_cuboid_mesh(fp, ht, cell))

    def free_fn(X, Y, slack=0.0):
        free = _dist_to_footprints(X, Y, fps) > clearance - slack
        if slack > 0.0:  # the route grid also covers the margin along the walls
            free &= ((X > clearance - slack) & (X < L[0] - clearance + slack) & (Y > clearance - slack)
                     & (Y < L[1] - clearance + slack))
        return free

    bounds = ((clearance, L[0] - clearance), (clearance, L[1] - clearance))
    poses, h = pose_grid(free_fn, bounds, K, rng, h0=h0)
    return mb.mesh(), poses, fps, heights, h, free_fn, bounds


# Tower base 55 cm across plus a 5 cm dilation: clearance from walls and
# obstacle footprints for tower poses.
TOWER_CLEARANCE = 0.275 + 0.05


def ward(seed: int = 1, cell: float = 0.1, K: int = 5000) -> Workload:
    """8 x 6 x 3 m ward: 6 beds (2 x 1 x 0.6 m) and 10 cuboids, every face
    gridded at ~0.1 m (~52k triangles); K poses on the free grid; tower lamp
    of 8 x 20 W sources at 0.2 ... 1.6 m."""
    rng = np.random.default_rng(seed)
    L = (8.0, 6.0, 3.0)
    mesh, poses, fps, heights, h, free_fn, bounds = _room_with_cuboids(rng, L, 6, 10, cell, TOWER_CLEARANCE, K)
    return Workload("ward", mesh, poses, tower_lamp(),
                    dict(seed=seed, room=L, cell=cell, pose_spacing=h, n_obstacles=len(fps)), free_fn, bounds)


def _room_tri_count(L, dims_list, h):
    return box_tri_count(L, h) + sum(box_tri_count(d, h) for d in dims_list)


def _cell_for_target(count_fn, target, lo=0.005, hi=3.0, iters=40):
    """Largest cell size whose triangle count is >= target (bisection)."""
    for _ in range(iters):
        mid = math.sqrt(lo * hi)
        if count_fn(mid) >= target:
            lo = mid
        else:
            hi = mid
    return lo


def batch_room(seed: int, n_range=(2000, 80000), k_range=(500, 8000)) -> Workload:
    """One room of the batched workload: Lx, Ly ~ U[3, 10] m, 3 m high, 2-16
    cuboids (edges ~ U[0.3, 1.2] m); target triangle count and pose count
    drawn log-uniform from n_range and k_range; cell size bisected to reach
    the triangle target; tower lamp."""
    rng = np.random.default_rng(seed)
    L = (float(rng.uniform(3.0, 10.0)), float(rng.uniform(3.0, 10.0)), 3.0)
    n_target = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
    K = int(round(math.exp(rng.uniform(math.log(k_range[0]), math.log(k_range[1])))))
    n_cub = int(rng.integers(2, 17))
    dims = [tuple(float(v) for v in rng.uniform(0.3, 1.2, size=3)) for _ in range(n_cub)]
    cell = _cell_for_target(lambda hh: _room_tri_count(L, dims, hh), n_target)
    mb = MeshBuilder()
    mb.add(*box_surface((0, 0, 0), L, [_ncells(l, cell) for l in L], inward=True))
    fps = []
    for dd in dims:
        fp = _place_cuboid(rng, (0, 0), L[:2], dd)
        fps.append(fp)
        mb.add(*_cuboid_mesh(fp, dd[2], cell))

    c = TOWER_CLEARANCE

    def free_fn(X, Y, slack=0.0):
        free = _dist_to_footprints(X, Y, fps) > c - slack
        if slack > 0.0:  # the route grid also covers the margin along the walls
            free &= (X > c - slack) & (X < L[0] - c + slack) & (Y > c - slack) & (Y < L[1] - c + slack)
        return free

    bounds = ((c, L[0] - c), (c, L[1] - c))
    poses, h = pose_grid(free_fn, bounds, K, rng, h0=0.25)
    return Workload(f"batch_room_{seed}", mb.mesh(), poses, tower_lamp(),
                    dict(seed=seed, room=L, cell=cell, pose_spacing=h, n_target=n_target, n_obstacles=n_cub),
                    free_fn, bounds)


def batch(seed: int = 3, n_rooms: int = 64, **kw) -> list:
    """Independent rooms of uneven size, room r seeded with seed + r."""
    return [batch_room(seed + r, **kw) for r in range(n_rooms)]


def floorplan(seed: int = 2, target_tris: int = 500_000, K: int = 20000) -> Workload:
    """12 rooms in a 4 x 3 slot grid (column widths and row depths ~ U[3, 10] m,
    3 m high) separated by 0.15 m walls, joined by 1.2 m x 2.1 m doorway
    tunnels on a seeded spanning tree of slot adjacencies; 5-20 cuboids per
    room; cell size bisected so the mesh has ~target_tris triangles; K poses;
    tower lamp."""
    rng = np.random.default_rng(seed)
    ncol, nrow, t, H = 4, 3, 0.15, 3.0
    DW, DH = 1.2, 2.1
    widths = rng.uniform(3.0, 10.0, size=ncol)
    depths = rng.uniform(3.0, 10.0, size=nrow)
    X0 = np.concatenate([[0.0], np.cumsum(widths + t)[:-1]])
    Y0 = np.concatenate([[0.0], np.cumsum(depths + t)[:-1]])
    rooms = {(c, r): (X0[c], X0[c] + widths[c], Y0[r], Y0[r] + depths[r]) for c in range(ncol) for r in range(nrow)}
    # seeded spanning tree (randomised Kruskal over slot adjacencies)
    edges = [((c, r), (c + 1, r)) for c in range(ncol - 1) for r in range(nrow)] + \
            [((c, r), (c, r + 1)) for c in range(ncol) for r in range(nrow - 1)]
    order = rng.permutation(len(edges))
    parent = {k: k for k in rooms}

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    doors = []  # (room_a, room_b, axis of the wall normal, centre along the wall)
    for e in order:
        a, b = edges[e]
        ra, rb = find(a), find(b)
        if ra == rb:
            continue
        parent[ra] = rb
        if a[1] == b[1]:  # neighbours along x: wall normal is x, door spans y
            y0, y1 = rooms[a][2], rooms[a][3]
            cen = float(rng.uniform(y0 + 0.9, y1 - 0.9))
            doors.append((a, b, 0, cen))
        else:             # neighbours along y: wall normal is y, door spans x
            x0, x1 = rooms[a][0], rooms[a][1]
            cen = float(rng.uniform(x0 + 0.9, x1 - 0.9))
            doors.append((a, b, 1, cen))
    furn = {}
    for key, (x0, x1, y0, y1) in rooms.items():
        n = int(rng.integers(5, 21))
        lst = []
        for _ in range(n):
            dims = tuple(float(v) for v in rng.uniform(0.3, 1.2, size=3))
            lst.append((_place_cuboid(rng, (x0, y0), (x1, y1), dims), dims[2]))
        furn[key] = lst

    def build(h, count_only=False):
        fs = None if count_only else FaceSet()
        count = 0

        def rect(axis, coord, ub, vb, sign, holes=()):
            nonlocal count
            if count_only:
                nu = sum(_ncells(ub[i + 1] - ub[i], h) for i in range(len(ub) - 1))
                nv = sum(_ncells(vb[i + 1] - vb[i], h) for i in range(len(vb) - 1))
                count += 2 * nu * nv  # holes are small; the count is an estimate
            else:
                fs.rect(axis, coord, ub, vb, h, sign, holes)

        for key, (x0, x1, y0, y1) in rooms.items():
            # floor (normal +z), ceiling (normal -z); rect(axis=2) has (b, c) = (x, y)
            rect(2, 0.0, [x0, x1], [y0, y1], +1)
            rect(2, H, [x0, x1], [y0, y1], -1)
            # walls: axis 0 (x = const) has (b, c) = (y, z); axis 1 (y = const) has (b, c) = (z, x)
            for axis, coord, sign in ((0, x0, +1), (0, x1, -1), (1, y0, +1), (1, y1, -1)):
                holes, breaks = [], []
                for (a, b, dax, cen) in doors:
                    if key not in (a, b) or dax != axis:
                        continue
                    lo_side = (key == a)  # room a is on the low side of the wall
                    if (lo_side and sign < 0) or (not lo_side and sign > 0):
                        breaks.append(cen)
                if axis == 0:
                    ub = [y0, y1]
                    vb = [0.0, H]
                    for cen in breaks:
                        ub = sorted(ub + [cen - DW / 2, cen + DW / 2])
                        vb = sorted(set(vb + [DH]))
                        holes.append((cen - DW / 2, cen + DW / 2, 0.0, DH))
                    rect(0, coord, ub, vb, sign, holes)
                else:
                    ub = [0.0, H]
                    vb = [x0, x1]
                    for cen in breaks:
                        vb = sorted(vb + [cen - DW / 2, cen + DW / 2])
                        ub = sorted(set(ub + [DH]))
                        holes.append((0.0, DH, cen - DW / 2, cen + DW / 2))
                    rect(1, coord, ub, vb, sign, holes)
        # doorway tunnels: two jambs, lintel and threshold, normals into the tunnel
        for (a, b, dax, cen) in doors:
            if dax == 0:
                xa, xb = rooms[a][1], rooms[b][0]
                u0, u1 = cen - DW / 2, cen + DW / 2
                # jambs at y = u0 (normal +y) and y = u1 (normal -y): axis 1, (b, c) = (z, x)
                rect(1, u0, [0.0, DH], [xa, xb], +1)
                rect(1, u1, [0.0, DH], [xa, xb], -1)
                # lintel at z = DH (normal -z) and threshold z = 0 (normal +z): axis 2, (x, y)
                rect(2, DH, [xa, xb], [u0, u1], -1)
                rect(2, 0.0, [xa, xb], [u0, u1], +1)
            else:
                ya, yb = rooms[a][3], rooms[b][2]
                u0, u1 = cen - DW / 2, cen + DW / 2
                # jambs at x = u0 (normal +x) and x = u1 (normal -x): axis 0, (b, c) = (y, z)
                rect(0, u0, [ya, yb], [0.0, DH], +1)
                rect(0, u1, [ya, yb], [0.0, DH], -1)
                rect(2, DH, [u0, u1], [ya, yb], -1)
                rect(2, 0.0, [u0, u1], [ya, yb], +1)
        for key, lst in furn.items():
            for fp, ht in lst:
                if count_only:
                    count += box_tri_count((fp.w, fp.d, ht), h)
                else:
                    fs.add_mesh(*_cuboid_mesh(fp, ht, h))
        return count if count_only else fs.mesh()

    cell = _cell_for_target(lambda hh: build(hh, count_only=True), target_tris, lo=0.01, hi=2.0, iters=30)
    mesh = build(cell)
    # free space: room interiors shrunk by the clearance, minus obstacle
    # footprints, plus doorway corridors through the wall gaps
    c = TOWER_CLEARANCE
    all_fp = [fp for lst in furn.values() for fp, _ in lst]

    def free_fn(X, Y, slack=0.0):
        cc = c - slack
        inside = np.zeros(X.shape, bool)
        for (x0, x1, y0, y1) in rooms.values():
            inside |= (X > x0 + cc) & (X < x1 - cc) & (Y > y0 + cc) & (Y < y1 - cc)
        for (a, b, dax, cen) in doors:
            if dax == 0:
                xa, xb = rooms[a][1], rooms[b][0]
                inside |= (X > xa - c - 1e-9) & (X < xb + c + 1e-9) & (Y > cen - DW / 2 + cc) & (Y < cen + DW / 2 - cc)
            else:
                ya, yb = rooms[a][3], rooms[b][2]
                inside |= (Y > ya - c - 1e-9) & (Y < yb + c + 1e-9) & (X > cen - DW / 2 + cc) & (X < cen + DW / 2 - cc)
        return inside & (_dist_to_footprints(X, Y, all_fp) > cc)

    ext = ((0.0, float(X0[-1] + widths[-1])), (0.0, float(Y0[-1] + depths[-1])))
    poses, h = pose_grid(free_fn, ext, K, rng, h0=0.25)
    return Workload("floorplan", mesh, poses, tower_lamp(),
                    dict(seed=seed, cell=cell, pose_spacing=h, n_doors=len(doors), n_obstacles=len(all_fp),
                         extent=ext), free_fn, ext)


CONFIGS = {
    "box_room": box_room,
    "ward": ward,
    "floorplan": floorplan,
}
