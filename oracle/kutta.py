"""Oracle: the Kutta condition as a constraint on a body's stream-function value.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Boundary Conditions" (its trailing-edge paragraph): where the flow must
leave a body at a given place, a point is added in the fluid such that the flow
leaves along the line from the body to that point; with the body held at one
constant stream-function value, the dividing streamline psi = psi_b then passes
through the point.

Reading applied here (the paper gives the idea in words only):

* for a body b with a Kutta point K_b, the equation psi(K_b) = psi_b replaces the
  body's zero-circulation equation (its summed row T^T K psi of the constrained
  system); psi_b stays one unknown shared by all the body's nodes.  Bodies
  without a Kutta point keep the zero-circulation row.  The body's circulation is
  then whatever the flow needs: the summed body row R_b = sum_{n in b} (K psi)_n
  equals the flux of grad psi through the body's ring of cells, i.e. the
  circulation around the body;
* K_b is the grid node nearest to the given point in undisplaced grid
  coordinates, i = floor((x - x0)/hx + 1/2) (ties to the larger index), likewise
  j; it must be a fluid node off the Dirichlet sides.  No node is repositioned:
  a caller who wants the point exactly places it on a grid node;
* the system is square and, with a Kutta row, no longer symmetric: it is solved
  directly by sparse LU, the plain definition of its solution.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import assemble
from .mesh import node_coords, spacing
from .solve import dirichlet_mask, dirichlet_values, selection_matrix


class KuttaError(ValueError):
    pass


def kutta_node(grid, point):
    """Node id j (nx+1) + i nearest to point (x, y) (undisplaced grid)."""
    hx, hy = spacing(grid)
    i = int(np.floor((point[0] - grid.x0) / hx + 0.5))
    j = int(np.floor((point[1] - grid.y0) / hy + 0.5))
    if not (0 <= i <= grid.nx and 0 <= j <= grid.ny):
        raise KuttaError("Kutta point outside the grid")
    return j * (grid.nx + 1) + i


@dataclass
class KuttaSolution:
    psi: np.ndarray          # nodal psi (body nodes carry psi_b)
    psi_b: np.ndarray        # (nbody,)
    body_rows: np.ndarray    # (nbody,) summed body rows R_b of K psi
    kutta_nodes: list        # node id per body, -1 for none
    nfree: int


def solve_kutta(mesh, flow, kutta_points, g=None):
    """Constrained solve with the Kutta rows.  kutta_points: one (x, y) or None per
    body.  g: optional full nodal vector overriding the Dirichlet data."""
    grid = mesh.grid
    nb = len(mesh.circles)
    if len(kutta_points) != nb:
        raise KuttaError("one Kutta point (or None) per body")
    K = assemble(mesh)
    if g is None:
        g = dirichlet_values(grid, flow, mesh.circles)
    dmask = dirichlet_mask(grid, flow).ravel()
    g = np.where(dmask, np.asarray(g, dtype=float).ravel(), 0.0)
    body = mesh.body.ravel().astype(np.int64)
    free = (~dmask) & (body < 0)
    dof = np.full(body.shape, -1, dtype=np.int64)
    nfree = int(free.sum())
    dof[free] = np.arange(nfree)
    dof[body >= 0] = nfree + body[body >= 0]
    ndof = nfree + nb
    T = selection_matrix(dof, ndof)
    A = (T.T @ K @ T).tolil()
    rhs = -(T.T @ (K @ g))
    knodes = []
    for b, pt in enumerate(kutta_points):
        if pt is None:
            knodes.append(-1)
            continue
        n = kutta_node(grid, pt)
        if dof[n] < 0 or dof[n] >= nfree:
            raise KuttaError("Kutta point must be a fluid node off the Dirichlet sides")
        knodes.append(n)
        r = nfree + b
        A.rows[r] = []
        A.data[r] = []
        A[r, dof[n]] = 1.0
        A[r, r] = -1.0
        rhs[r] = 0.0
    y = spla.splu(sp.csc_matrix(A)).solve(rhs) if ndof > 0 else np.zeros(0)
    psi = g + T @ y
    Kpsi = K @ psi
    rows = np.array([Kpsi[body == b].sum() for b in range(nb)])
    return KuttaSolution(psi, y[nfree:].copy(), rows, knodes, nfree)


def lifting_cylinder_psi(X, Y, U, centre, a, gamma):
    """Stream function of uniform flow U past a cylinder of radius a at centre with
    circulation gamma (counter-clockwise positive):
    psi = U y' (1 - a^2 / r^2) - gamma / (2 pi) ln(r / a), (x', y') = (X, Y) - centre.
    Zero on the cylinder."""
    x = np.asarray(X, dtype=float) - centre[0]
    y = np.asarray(Y, dtype=float) - centre[1]
    r2 = x * x + y * y
    with np.errstate(divide="ignore", invalid="ignore"):  # the centre itself: no value
        return U * y * (1.0 - a * a / r2) - gamma / (2.0 * np.pi) * np.log(np.sqrt(r2) / a)


def circulation_through(point, U, centre, a):
    """The circulation for which the zero streamline of lifting_cylinder_psi passes
    through point (outside the cylinder, off its horizontal axis)."""
    x = point[0] - centre[0]
    y = point[1] - centre[1]
    r = np.hypot(x, y)
    return 2.0 * np.pi * U * y * (1.0 - a * a / (r * r)) / np.log(r / a)


def mixed_solve_kutta(mm, flow, kutta_points, g=None):
    """The Kutta rows on the mixed-cell mesh: as solve_kutta, with the mixed mesh's
    unknowns (background fluid nodes of some element off the Dirichlet sides, one
    psi_b per body for all its cut points).  Returns a KuttaSolution over the mixed
    nodes (inside nodes 0; body_rows summed over each body's cut points)."""
    from .mixed import assemble_mixed
    grid = mm.grid
    nb = len(mm.circles)
    if len(kutta_points) != nb:
        raise KuttaError("one Kutta point (or None) per body")
    N = grid.nodes
    n = mm.n_nodes
    K = assemble_mixed(mm)
    if g is None:
        g = np.concatenate([dirichlet_values(grid, flow, mm.circles), np.zeros(len(mm.pxy))])
    dmask = np.concatenate([dirichlet_mask(grid, flow).ravel() & (mm.body.ravel() < 0),
                            np.zeros(len(mm.pxy), bool)])
    g = np.where(dmask, np.asarray(g, dtype=float), 0.0)
    used = np.zeros(n, bool)
    used[mm.elem_nodes[mm.elem_nodes >= 0]] = True
    free = used & ~dmask
    free[N:] = False
    dof = np.full(n, -1, dtype=np.int64)
    nfree = int(free.sum())
    dof[free] = np.arange(nfree)
    dof[N:] = nfree + mm.pbody
    ndof = nfree + nb
    T = selection_matrix(dof, ndof)
    A = (T.T @ K @ T).tolil()
    rhs = -(T.T @ (K @ g))
    knodes = []
    for b, pt in enumerate(kutta_points):
        if pt is None:
            knodes.append(-1)
            continue
        kn = kutta_node(grid, pt)
        if dof[kn] < 0 or dof[kn] >= nfree:
            raise KuttaError("Kutta point must be a fluid node of the mesh off the "
                             "Dirichlet sides")
        knodes.append(kn)
        r = nfree + b
        A.rows[r] = []
        A.data[r] = []
        A[r, dof[kn]] = 1.0
        A[r, r] = -1.0
        rhs[r] = 0.0
    y = spla.splu(sp.csc_matrix(A)).solve(rhs) if ndof > 0 else np.zeros(0)
    psi = g + T @ y
    Kpsi = K @ psi
    rows = np.array([Kpsi[N:][mm.pbody == b].sum() for b in range(nb)])
    return KuttaSolution(psi, y[nfree:].copy(), rows, knodes, nfree)
