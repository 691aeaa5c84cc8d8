"""Oracle: body-conforming Q1 mesh from a Cartesian grid and a list of circles.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper's section "Body-Conforming Grid Generation":

1. a uniform Cartesian background grid covers the domain;
2. grid points just inside each immersed body are moved onto the body
   surface, with displacement d_ik = x_ik - x_gk;
3. the displacements are propagated into the domain by the Laplace equation
   for d, with d = d_i on the body and d = 0 on the outer boundaries, and the
   vertices are moved by x_new = x_old + d.

Readings applied here (the paper leaves these open or describes a mesher with
mixed cells that is not built):

* the background quad topology is kept: no node splitting, no triangles or
  pentagons;
* "just inside" = a body node with at least one fluid node among its eight
  neighbours (3x3 block); such a node is "snapped";
* projection is radial (closest point on the circle): p = c + (r/rho)(x - c);
* a node exactly on a circle counts as inside (<=);
* the Laplace problem for d is not solved to convergence: a fixed number of
  Jacobi sweeps (200 by default) of the five-point average
  d <- wx (d_E + d_W) + wy (d_N + d_S), with wx = hy^2 / (2 (hx^2 + hy^2)) and
  wy = hx^2 / (2 (hx^2 + hy^2)), evaluated in exactly that order, is applied to
  fluid nodes off the outer boundary.  Snapped nodes keep their projection
  displacement; outer-boundary nodes and deep body nodes keep d = 0;
* the minimum-spacing redistribution of boundary points is omitted (no rule
  is given).

Array convention: node arrays have shape (ny+1, nx+1) indexed [j, i]; the
flat node id is j*(nx+1) + i (x fastest).  Displacements have shape
(2, ny+1, nx+1): component 0 is x, component 1 is y.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

FLUID, SNAPPED, DEEP = 0, 1, 2


class GeometryError(ValueError):
    """Input geometry rejected (overlap, too close to the outer boundary, or a
    circle under-resolved by the grid)."""


def spacing(grid):
    """Cell sizes hx = (x1 - x0)/nx, hy = (y1 - y0)/ny."""
    return (grid.x1 - grid.x0) / grid.nx, (grid.y1 - grid.y0) / grid.ny


def node_coords(grid):
    """Background node coordinates x_i = x0 + i hx, y_j = y0 + j hy as
    (ny+1, nx+1) arrays."""
    hx, hy = spacing(grid)
    xs = grid.x0 + np.arange(grid.nx + 1, dtype=np.float64) * hx
    ys = grid.y0 + np.arange(grid.ny + 1, dtype=np.float64) * hy
    X = np.broadcast_to(xs[None, :], (grid.ny + 1, grid.nx + 1)).copy()
    Y = np.broadcast_to(ys[:, None], (grid.ny + 1, grid.nx + 1)).copy()
    return X, Y


def _real(v):
    return float(np.real(v))


def check_geometry(grid, circles, max_bodies=64):
    """Reject inputs the conforming rule cannot mesh.

    * at most ``max_bodies`` circles;
    * every radius r >= 2 max(hx, hy);
    * every circle at least one cell away from each outer side;
    * circles pairwise disjoint (centre distance strictly above r_a + r_b).
    """
    hx, hy = spacing(grid)
    if grid.nx < 2 or grid.ny < 2:
        raise GeometryError("grid needs at least 2x2 cells")
    if len(circles) > max_bodies:
        raise GeometryError("too many bodies")
    h = max(hx, hy)
    for (cx, cy, r) in circles:
        cx, cy, r = _real(cx), _real(cy), _real(r)
        if not (r >= 2.0 * h):
            raise GeometryError("circle radius below two cells")
        if not (cx - r >= grid.x0 + hx and cx + r <= grid.x1 - hx and
                cy - r >= grid.y0 + hy and cy + r <= grid.y1 - hy):
            raise GeometryError("circle within one cell of the outer boundary")
    for a in range(len(circles)):
        for b in range(a + 1, len(circles)):
            ax, ay, ar = (_real(v) for v in circles[a])
            bx, by, br = (_real(v) for v in circles[b])
            dx, dy = ax - bx, ay - by
            if not (dx * dx + dy * dy > (ar + br) * (ar + br)):
                raise GeometryError("circles overlap")


def classify(grid, circles):
    """Node kinds and body ids.

    Body b holds the nodes with (x - cx)^2 + (y - cy)^2 <= r^2 (plain FP64,
    no fused multiply-add).  A body node is SNAPPED when any of its eight
    neighbours is a fluid node, DEEP otherwise.  Returns (kind, body) int8
    arrays of shape (ny+1, nx+1); body is -1 for fluid nodes.
    """
    X, Y = node_coords(grid)
    body = np.full(X.shape, -1, dtype=np.int8)
    for b, (cx, cy, r) in enumerate(circles):
        cx, cy, r = _real(cx), _real(cy), _real(r)
        dx = X - cx
        dy = Y - cy
        inside = (dx * dx + dy * dy) <= r * r
        body[inside] = b
    isbody = body >= 0
    fluid = ~isbody
    # any fluid node in the 3x3 block around each node
    pad = np.pad(fluid, 1, constant_values=False)
    near_fluid = np.zeros_like(fluid)
    ny1, nx1 = fluid.shape
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            near_fluid |= pad[1 + dj:1 + dj + ny1, 1 + di:1 + di + nx1]
    kind = np.full(X.shape, FLUID, dtype=np.int8)
    kind[isbody & near_fluid] = SNAPPED
    kind[isbody & ~near_fluid] = DEEP
    return kind, body


def snap_displacement(grid, circles, kind, body):
    """Displacement of each snapped node to its radial projection on the
    circle (d_ik = x_ik - x_gk), zero elsewhere.

    The projection is s = r / rho, p = c + s (x - c), d = p - x, with
    rho = sqrt((x - cx)^2 + (y - cy)^2), in that order of operations.
    Circle parameters may be complex (complex-step differentiation); the
    classification is passed in and therefore frozen.
    """
    X, Y = node_coords(grid)
    dtype = np.result_type(np.float64, *[np.asarray(v) for c in circles for v in c])
    d = np.zeros((2,) + X.shape, dtype=dtype)
    for b, (cx, cy, r) in enumerate(circles):
        sel = (kind == SNAPPED) & (body == b)
        x = X[sel]
        y = Y[sel]
        dx = x - cx
        dy = y - cy
        rho = np.sqrt(dx * dx + dy * dy)
        s = r / rho
        px = cx + s * dx
        py = cy + s * dy
        d[0][sel] = px - x
        d[1][sel] = py - y
    return d


def jacobi_weights(grid):
    """wx = hy^2 / (2 (hx^2 + hy^2)), wy = hx^2 / (2 (hx^2 + hy^2))."""
    hx, hy = spacing(grid)
    s = 2.0 * (hx * hx + hy * hy)
    return (hy * hy) / s, (hx * hx) / s


def update_mask(kind):
    """Nodes moved by the smoother: fluid nodes off the outer boundary."""
    upd = kind == FLUID
    upd[0, :] = False
    upd[-1, :] = False
    upd[:, 0] = False
    upd[:, -1] = False
    return upd


def smooth(grid, kind, d0, nsweeps):
    """Jacobi sweeps of the displacement Laplace equation.

    Every sweep evaluates d_new = wx (d_E + d_W) + wy (d_N + d_S) from the
    previous sweep's values at all update nodes; all other nodes keep their
    value.  Works on real or complex arrays.
    """
    wx, wy = jacobi_weights(grid)
    upd = update_mask(kind)
    d = d0.copy()
    for _ in range(nsweeps):
        new = d.copy()
        east = d[:, 1:-1, 2:]
        west = d[:, 1:-1, :-2]
        north = d[:, 2:, 1:-1]
        south = d[:, :-2, 1:-1]
        new[:, 1:-1, 1:-1] = wx * (east + west) + wy * (north + south)
        d = np.where(upd[None], new, d)
    return d


def cell_nodes(grid):
    """Flat node ids of every cell's four nodes in counter-clockwise order
    (i,j), (i+1,j), (i+1,j+1), (i,j+1); shape (ny*nx, 4), cell id j*nx + i."""
    nx, ny = grid.nx, grid.ny
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    n0 = (j * (nx + 1) + i).ravel()
    return np.stack([n0, n0 + 1, n0 + nx + 2, n0 + nx + 1], axis=1)


def active_cells(grid, body):
    """A cell is active unless its four nodes all belong to the same body."""
    cn = cell_nodes(grid)
    b = body.ravel()[cn].astype(np.int32)
    same = (b[:, 0] >= 0) & (b[:, 1] == b[:, 0]) & (b[:, 2] == b[:, 0]) & (b[:, 3] == b[:, 0])
    return ~same


@dataclass
class Mesh:
    grid: object
    circles: list
    kind: np.ndarray   # (ny+1, nx+1) int8: FLUID / SNAPPED / DEEP
    body: np.ndarray   # (ny+1, nx+1) int8: body id or -1
    disp: np.ndarray   # (2, ny+1, nx+1) float64 (or complex128)

    def coords(self):
        X, Y = node_coords(self.grid)
        return X + self.disp[0], Y + self.disp[1]


def conform(grid, circles, nsweeps=200, kind_body=None):
    """Full mesh rule: check, classify, snap, smooth.

    ``kind_body`` freezes the classification (used by complex-step and finite
    differences); otherwise it is computed from the (real) circles.
    """
    check_geometry(grid, circles)
    if kind_body is None:
        kind, body = classify(grid, circles)
    else:
        kind, body = kind_body
    d0 = snap_displacement(grid, circles, kind, body)
    d = smooth(grid, kind, d0, nsweeps)
    return Mesh(grid, list(circles), kind, body, d)
