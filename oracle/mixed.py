"""Oracle: the paper's mixed-cell body-conforming mesh and the stream-function
solve on it.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Body-Conforming Grid Generation" describes a mesher whose cells near a
body become triangles, quadrilaterals and pentagons: grid points just inside a
body are moved onto it along the grid lines, a point that meets the boundary in
two places is split (a "node-splitting event"), and each pentagon is cut into a
triangle and a quadrilateral (points 1, 2 -> a, b forming a triangle with node 3;
node 10 split into e, f, pentagon e-9-8-11-f cut into e-9-8 and e-8-11-f).  The
figure that shows it is missing; the reading implemented here (every step is
listed with the passage it follows):

1. classification as for the quadrilateral mesher: a node is inside body b when
   (x - cx)^2 + (y - cy)^2 <= r^2 (FP64);
2. cut points: every grid edge that joins an inside node I to a fluid node O is
   cut where it meets the circle, P = I + t (O - I) with the root t in [0, 1) of
   |I - c + t (O - I)|^2 = r^2.  The inside node is moved onto the body along
   that grid line: d_ik = P - I.  An inside node with fluid neighbours in k
   directions gives k boundary points (k >= 2: the node is split);
3. the displacements are propagated with the Jacobi sweeps of the quadrilateral
   mesher (d <- wx (d_E + d_W) + wy (d_N + d_S) on fluid nodes off the outer
   boundary, outer nodes fixed at 0), where an inside neighbour contributes the
   displacement of the cut point on the shared edge;
4. cells: a cell with four fluid corners stays a quadrilateral (corners
   displaced); a cell with four inside corners of one body is not meshed; any
   other cell becomes the polygon met by walking its boundary counter-clockwise
   from corner (i, j): fluid corners and the cut points of its cut edges.  One
   fluid corner gives a triangle, two adjacent ones a quadrilateral, three a
   pentagon, cut into the triangle (p_a, c_k+1, c_k+2) and the quadrilateral
   (p_a, c_k+2, c_k+3, p_b), where c_k is the inside corner and p_a, p_b the cut
   points after and before it in counter-clockwise order (the paper's e-9-8 and
   e-8-11-f).  A triangle whose two cut points lie within 1e-12 max(hx, hy) of
   each other (max norm: its fluid corner lies on the circle to rounding and both
   cut edges meet the circle there) is a sliver of no area and is not meshed: the
   smallest case of the paper's minimum spacing of boundary points, which changes
   the equations by O(1e-12 h);
5. a cell whose inside and fluid corners alternate around it (a thin part of a
   body, a trailing edge above all, crosses it diagonally; impossible for a circle
   of radius >= 2h) has two separate fluid parts: each fluid corner k gets the
   triangle (cut point of edge k-1, corner k, cut point of edge k), in corner
   order, each subject to the sliver rule -- the corner treatment of section
   "Boundary Conditions" read as node splitting of the inside corners;
   inputs this reading cannot mesh are rejected (GeometryError): besides the
   quadrilateral mesher's checks, a grid edge or cell whose nodes lie in two
   different bodies;
6. elements: triangles are linear (P1, exact integral), quadrilaterals bilinear
   (Q1, 2x2 Gauss) as in section "Weak formulation"; beyond the sliver rule of
   step 4 the paper's minimum-spacing redistribution of boundary points is omitted
   (no rule is given).

The stream-function problem is the quadrilateral mesh's: every cut point of body
b carries the one unknown psi_b, fluid nodes are free or Dirichlet by the side
boundary conditions; the reduced system A y = b is solved by sparse LU.

Node numbering of a mixed mesh: background nodes j (nx+1) + i first (inside ones
unused), then the cut points in edge order: horizontal edges (i, j)-(i+1, j) by
j nx + i, then vertical edges (i, j)-(i, j+1) by j (nx+1) + i.  Elements are
ordered by cell id, a pentagon's triangle before its quadrilateral.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import (GeometryError, check_geometry, spacing, node_coords, jacobi_weights, FLUID,
                   SNAPPED, DEEP)
from .airfoil import Circle
from .fem import element_stiffness
from .solve import dirichlet_values, dirichlet_mask


# Cut points of a triangle closer than SLIVER * max(hx, hy) (max norm) make a sliver
# that is not meshed.
SLIVER = 1e-12


def triangle_stiffness(xe, ye):
    """P1 stiffness of triangles with vertex coordinates of shape (..., 3):
    K_ab = (b_a b_b + c_a c_b) / (4 A), b_a = y_(a+1) - y_(a+2),
    c_a = x_(a+2) - x_(a+1), 2 A = sum_a b_a x_a."""
    xe = np.asarray(xe, dtype=float)
    ye = np.asarray(ye, dtype=float)
    b = np.roll(ye, -1, -1) - np.roll(ye, -2, -1)
    c = np.roll(xe, -2, -1) - np.roll(xe, -1, -1)
    twoA = (b * xe).sum(-1)
    return (b[..., :, None] * b[..., None, :] + c[..., :, None] * c[..., None, :]) / (
        2.0 * twoA[..., None, None])


def polygon_area(x, y):
    """Signed area (shoelace), counter-clockwise positive."""
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def _edge_root(ux, uy, vx, vy, r):
    """t in [0, 1) with |u + t v| = r, for |u| <= r < |u + v| (v along one axis)."""
    vv = vx * vx + vy * vy
    uv = ux * vx + uy * vy
    uu = ux * ux + uy * uy
    return (-uv + np.sqrt(uv * uv - vv * (uu - r * r))) / vv


@dataclass
class MixedMesh:
    grid: object
    circles: list
    kind: np.ndarray        # (ny+1, nx+1) as classify
    body: np.ndarray        # (ny+1, nx+1) body id or -1
    disp: np.ndarray        # (2, ny+1, nx+1) smoothed displacement of fluid nodes
    hpt: np.ndarray         # (ny+1, nx) index of the cut point of horizontal edge, -1
    vpt: np.ndarray         # (ny, nx+1) index of the cut point of vertical edge, -1
    pxy: np.ndarray         # (m, 2) cut point coordinates
    pbody: np.ndarray       # (m,) body of each cut point
    elem_nodes: np.ndarray  # (ne, 4) node ids (mixed numbering), -1 past nne
    elem_nne: np.ndarray    # (ne,) 3 or 4
    elem_cell: np.ndarray   # (ne,) cell id

    @property
    def n_nodes(self):
        return self.grid.nodes + len(self.pxy)

    def coords(self):
        """(x, y) of every mixed node: displaced background nodes, then cut points."""
        X, Y = node_coords(self.grid)
        x = np.concatenate([(X + self.disp[0]).ravel(), self.pxy[:, 0]])
        y = np.concatenate([(Y + self.disp[1]).ravel(), self.pxy[:, 1]])
        return x, y


def classify_bodies(grid, bodies):
    """Body of every node (the last body whose contains() holds, -1 for fluid) and
    the node kinds of the Q1 mesh's rule (a body node with a fluid node among its
    eight neighbours is SNAPPED, else DEEP).  Returns (kind, body), (ny+1, nx+1)."""
    X, Y = node_coords(grid)
    body = np.full(X.shape, -1, dtype=np.int8)
    for b, bd in enumerate(bodies):
        body[bd.contains(X, Y)] = b
    isbody = body >= 0
    fluid = ~isbody
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


def cut_points(grid, bodies, body):
    """Cut points of the grid edges that join an inside node to a fluid node (step 2),
    each from its body's cut(): for a circle the root t in [0, 1) of
    |I + t (O - I) - c| = r.  Returns (hpt, vpt, pxy, pbody)."""
    hx, hy = spacing(grid)
    X, Y = node_coords(grid)
    nx, ny = grid.nx, grid.ny
    hpt = np.full((ny + 1, nx), -1, dtype=np.int64)
    vpt = np.full((ny, nx + 1), -1, dtype=np.int64)
    pts, pb = [], []
    # horizontal edges in edge order, then vertical edges
    for horizontal in (True, False):
        if horizontal:
            ba, bb = body[:, :-1], body[:, 1:]
        else:
            ba, bb = body[:-1, :], body[1:, :]
        if np.any((ba >= 0) & (bb >= 0) & (ba != bb)):
            raise GeometryError("a grid edge joins two bodies")
        cut = (ba >= 0) != (bb >= 0)
        js, is_ = np.nonzero(cut)
        for j, i in zip(js, is_):
            a = (j, i)
            c = (j, i + 1) if horizontal else (j + 1, i)
            inside, outside = (a, c) if body[a] >= 0 else (c, a)
            b = int(body[inside])
            pts.append(bodies[b].cut(X[inside], Y[inside], X[outside], Y[outside]))
            pb.append(b)
            (hpt if horizontal else vpt)[j, i] = len(pts) - 1
    pxy = np.array(pts, dtype=float).reshape(-1, 2)
    return hpt, vpt, pxy, np.array(pb, dtype=np.int64)


def smooth_mixed(grid, body, hpt, vpt, pxy, nsweeps):
    """Jacobi sweeps of the displacement on fluid nodes (step 3).  The neighbour of
    a fluid node across a cut edge contributes d = P - I of that edge's cut point."""
    X, Y = node_coords(grid)
    nx, ny = grid.nx, grid.ny
    wx, wy = jacobi_weights(grid)
    fluid = body < 0
    upd = fluid.copy()
    upd[0, :] = upd[-1, :] = False
    upd[:, 0] = upd[:, -1] = False

    def across(idx, ni, nj, mask):
        """Displacement (P - I) of the cut point idx[mask] for the inside neighbour at
        (nj, ni) of every fluid node in mask; zeros elsewhere."""
        out = np.zeros((2, ny + 1, nx + 1))
        k = idx[mask]
        out[0][mask] = pxy[k, 0] - X[nj[mask], ni[mask]]
        out[1][mask] = pxy[k, 1] - Y[nj[mask], ni[mask]]
        return out

    J, I = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    inside = body >= 0
    # fluid node with an inside neighbour in each direction, and that edge's cut point
    e_in = np.zeros_like(fluid)
    e_in[:, :-1] = fluid[:, :-1] & inside[:, 1:]
    w_in = np.zeros_like(fluid)
    w_in[:, 1:] = fluid[:, 1:] & inside[:, :-1]
    n_in = np.zeros_like(fluid)
    n_in[:-1, :] = fluid[:-1, :] & inside[1:, :]
    s_in = np.zeros_like(fluid)
    s_in[1:, :] = fluid[1:, :] & inside[:-1, :]
    h_e = np.full((ny + 1, nx + 1), -1)
    h_e[:, :-1] = hpt
    h_w = np.full((ny + 1, nx + 1), -1)
    h_w[:, 1:] = hpt
    v_n = np.full((ny + 1, nx + 1), -1)
    v_n[:-1, :] = vpt
    v_s = np.full((ny + 1, nx + 1), -1)
    v_s[1:, :] = vpt
    east = across(h_e, I + 1, J, e_in)
    west = across(h_w, I - 1, J, w_in)
    north = across(v_n, I, J + 1, n_in)
    south = across(v_s, I, J - 1, s_in)
    d = np.zeros((2, ny + 1, nx + 1))
    for _ in range(nsweeps):
        dE = np.zeros_like(d)
        dW = np.zeros_like(d)
        dN = np.zeros_like(d)
        dS = np.zeros_like(d)
        dE[:, :, :-1] = d[:, :, 1:]
        dW[:, :, 1:] = d[:, :, :-1]
        dN[:, :-1, :] = d[:, 1:, :]
        dS[:, 1:, :] = d[:, :-1, :]
        dE = np.where(e_in[None], east, dE)
        dW = np.where(w_in[None], west, dW)
        dN = np.where(n_in[None], north, dN)
        dS = np.where(s_in[None], south, dS)
        new = wx * (dE + dW) + wy * (dN + dS)
        d = np.where(upd[None], new, d)
    return d


def _cell_polygons(grid, body, hpt, vpt, pxy):
    """Elements of every cell (step 4): list of (cell id, node ids)."""
    nx, ny = grid.nx, grid.ny
    hmax = max(spacing(grid))
    N = grid.nodes
    out = []
    for j in range(ny):
        for i in range(nx):
            corners = [(j, i), (j, i + 1), (j + 1, i + 1), (j + 1, i)]
            ins = [body[c] >= 0 for c in corners]
            cid = j * nx + i
            ids = [c[0] * (nx + 1) + c[1] for c in corners]
            if not any(ins):
                out.append((cid, ids))
                continue
            bs = {int(body[c]) for c in corners if body[c] >= 0}
            if len(bs) > 1:
                raise GeometryError("a cell touches two bodies")
            if all(ins):
                continue
            # cut point of the edge from corner k to corner k+1 (CCW)
            def edge_point(k):
                if k == 0:
                    return N + hpt[j, i]
                if k == 1:
                    return N + vpt[j, i + 1]
                if k == 2:
                    return N + hpt[j + 1, i]
                return N + vpt[j, i]
            poly = []
            for k in range(4):
                if not ins[k]:
                    poly.append(ids[k])
                if ins[k] != ins[(k + 1) % 4]:
                    poly.append(edge_point(k))
            nf = 4 - sum(ins)
            changes = sum(ins[k] != ins[(k + 1) % 4] for k in range(4))
            if changes == 4:
                # two fluid parts: a triangle at each fluid corner
                for k in range(4):
                    if ins[k]:
                        continue
                    pa, pb = edge_point((k + 3) % 4), edge_point(k)
                    gap = np.abs(pxy[pa - N] - pxy[pb - N]).max()
                    if not gap < SLIVER * hmax:
                        out.append((cid, [pa, ids[k], pb]))
                continue
            if nf == 1:
                # a triangle whose two cut points (nearly) coincide is a sliver of no
                # area (its fluid corner lies on the circle to rounding): not meshed
                pts = [q - N for q in poly if q >= N]
                gap = np.abs(pxy[pts[0]] - pxy[pts[1]]).max()
                if not gap < SLIVER * hmax:
                    out.append((cid, poly))
            elif nf == 2:
                out.append((cid, poly))
            else:  # pentagon: split at the point after the inside corner
                kin = ins.index(True)
                pa = edge_point(kin)
                pb = edge_point((kin + 3) % 4)
                c1, c2, c3 = ids[(kin + 1) % 4], ids[(kin + 2) % 4], ids[(kin + 3) % 4]
                out.append((cid, [pa, c1, c2]))
                out.append((cid, [pa, c2, c3, pb]))
    return out


def mixed_mesh(grid, circles, nsweeps=200):
    """Steps 1-5: the mixed-cell mesh of circles (cx, cy, r)."""
    return mixed_mesh_bodies(grid, [Circle(float(cx), float(cy), float(r))
                                    for cx, cy, r in circles], nsweeps)


def mixed_mesh_bodies(grid, bodies, nsweeps=200):
    """The mixed-cell mesh of bodies with contains() and cut() (circles, airfoils).
    The geometry checks use each body's bounding circle, which the mesh also keeps
    (its centre is the reference point of the surface-sample angles)."""
    circles = [bd.bounding_circle() for bd in bodies]
    check_geometry(grid, circles)
    kind, body = classify_bodies(grid, bodies)
    hpt, vpt, pxy, pbody = cut_points(grid, bodies, body)
    for b in range(len(bodies)):
        if not np.any(pbody == b):
            raise GeometryError(f"body {b} holds no grid node: the grid does not resolve it")
    d = smooth_mixed(grid, body, hpt, vpt, pxy, nsweeps)
    polys = _cell_polygons(grid, body, hpt, vpt, pxy)
    ne = len(polys)
    en = np.full((ne, 4), -1, dtype=np.int64)
    nne = np.zeros(ne, dtype=np.int64)
    ec = np.zeros(ne, dtype=np.int64)
    for e, (cid, ids) in enumerate(polys):
        en[e, :len(ids)] = ids
        nne[e] = len(ids)
        ec[e] = cid
    return MixedMesh(grid, list(circles), kind, body, d, hpt, vpt, pxy, pbody, en, nne, ec)


def element_matrices(mm):
    """K_e of every element (ne, 4, 4); triangles fill the leading 3 x 3 block."""
    x, y = mm.coords()
    ne = len(mm.elem_nne)
    K = np.zeros((ne, 4, 4))
    tri = mm.elem_nne == 3
    quad = ~tri
    if tri.any():
        n3 = mm.elem_nodes[tri, :3]
        K[tri, :3, :3] = triangle_stiffness(x[n3], y[n3])
    if quad.any():
        n4 = mm.elem_nodes[quad]
        K[quad] = element_stiffness(x[n4], y[n4])
    return K


def element_areas(mm):
    x, y = mm.coords()
    out = np.zeros(len(mm.elem_nne))
    for e in range(len(out)):
        ids = mm.elem_nodes[e, :mm.elem_nne[e]]
        out[e] = polygon_area(x[ids], y[ids])
    return out


def assemble_mixed(mm):
    """Assembled stiffness over all elements (CSR, mixed nodes)."""
    K = element_matrices(mm)
    rows, cols, vals = [], [], []
    for e in range(len(mm.elem_nne)):
        k = mm.elem_nne[e]
        ids = mm.elem_nodes[e, :k]
        rows.append(np.repeat(ids, k))
        cols.append(np.tile(ids, k))
        vals.append(K[e, :k, :k].ravel())
    n = mm.n_nodes
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


@dataclass
class MixedSolution:
    psi: np.ndarray     # (n_nodes,) mixed-node values (inside background nodes: 0)
    psi_b: np.ndarray   # (nbody,)
    nfree: int
    ndof: int
    A: object
    b: np.ndarray
    dof: np.ndarray


def mixed_solve(mm, flow, g=None, body_fixed=None):
    """Constrained stream-function solve on the mixed mesh.  ``g`` (full mixed-node
    vector) overrides the Dirichlet data; ``body_fixed`` (full mixed-node vector)
    prescribes every cut point instead of the body constraint (patch test)."""
    grid = mm.grid
    nb = len(mm.circles)
    N = grid.nodes
    n = mm.n_nodes
    K = assemble_mixed(mm)
    if g is None:
        g = np.concatenate([dirichlet_values(grid, flow, mm.circles), np.zeros(len(mm.pxy))])
    g = np.array(g, dtype=float)
    dmask = np.concatenate([dirichlet_mask(grid, flow).ravel() & (mm.body.ravel() < 0),
                            np.zeros(len(mm.pxy), bool)])
    used = np.zeros(n, bool)
    used[mm.elem_nodes[mm.elem_nodes >= 0]] = True
    if body_fixed is not None:
        g[N:] = np.asarray(body_fixed, dtype=float)[N:]
        dmask[N:] = True
        nb = 0
    g = np.where(dmask, g, 0.0)
    free = used & ~dmask
    free[N:] = False
    dof = np.full(n, -1, dtype=np.int64)
    nfree = int(free.sum())
    dof[free] = np.arange(nfree)
    if nb > 0:
        dof[N:] = nfree + mm.pbody
    ndof = nfree + nb
    rows = np.flatnonzero(dof >= 0)
    T = sp.csr_matrix((np.ones(rows.size), (rows, dof[rows])), shape=(n, ndof))
    A = (T.T @ K @ T).tocsc()
    b = -(T.T @ (K @ g))
    y = spla.splu(A).solve(b) if ndof > 0 else np.zeros(0)
    psi = g + T @ y
    return MixedSolution(psi, y[nfree:].copy(), nfree, ndof, A, b, dof)


def mixed_surface_samples(mm, psi, psi_b):
    """u_t = (psi_c - psi_b) / d_nc on every element edge that joins two cut points
    of the same body (the body surface segment of a cut cell): psi_c the mean of the
    element's vertex values, d_nc the distance from the vertex mean to the line
    through the edge, theta the polar angle of the edge midpoint.  Ordered by (body,
    element, local edge)."""
    x, y = mm.coords()
    N = mm.grid.nodes
    keys, th, ut = [], [], []
    for e in range(len(mm.elem_nne)):
        k = mm.elem_nne[e]
        ids = mm.elem_nodes[e, :k]
        gx, gy = x[ids].mean(), y[ids].mean()
        pc = psi[ids].mean()
        for a in range(k):
            p, q = ids[a], ids[(a + 1) % k]
            if p < N or q < N:
                continue
            b = int(mm.pbody[p - N])
            if int(mm.pbody[q - N]) != b:
                continue
            ex, ey = x[q] - x[p], y[q] - y[p]
            L = np.hypot(ex, ey)
            if L <= 1e-12 * max(spacing(mm.grid)):
                continue
            dnc = abs(ex * (gy - y[p]) - ey * (gx - x[p])) / L
            cx, cy, _ = mm.circles[b]
            th.append(np.arctan2(0.5 * (y[p] + y[q]) - cy, 0.5 * (x[p] + x[q]) - cx))
            ut.append((pc - psi_b[b]) / dnc)
            keys.append((b, e, a))
    order = sorted(range(len(keys)), key=lambda i: keys[i])
    return (np.array(th)[order], np.array(ut)[order],
            np.array([keys[i][0] for i in order], dtype=np.int8))
