"""Oracle: constrained stream-function solve and post-processing.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (sections "Boundary Conditions", "Weak formulation",
"Matrix-Free Conjugate Gradient with Multiple Constraint Enforcement" and
Algorithm 1 of the appendix):

* psi is a Q1 field; Dirichlet nodes carry prescribed values g; every node of
  body b carries the single unknown psi_b (constant-streamline condition
  psi = C_i on each body, with C_i unknown); all other nodes -- interior and
  natural-boundary nodes (zero flux, f_e^(N) = 0) -- are free.
* The unknowns are y = [free nodal values; psi_b for each body], so
  N_dof = N_int + N_N + N_b.  With the selection matrix T (node -> unknown)
  and the lifting g, psi = g + T y.
* Algorithm 1 sums each element residual into the free-node entries and, for
  body nodes, into one entry per body.  That is T^T applied to K psi, so the
  equations it drives to zero are  T^T K (g + T y) = 0, i.e. the symmetric
  positive definite system  A y = b  with  A = T^T K T  and  b = -T^T K g.
  The CG iteration of Algorithm 1 converges to the solution of this system;
  the oracle solves it directly (sparse LU), which is the plain definition of
  the answer.

Readings applied here:

* boundary data: a side with code 1 carries psi = U y, code 2 carries the
  isolated-cylinder stream function psi = U (y - cy)(1 - a^2 / rho^2) about
  body 0, code 0 is natural (codes 3 and 4 are the potential's: U x and the
  isolated-cylinder potential U (x - cx)(1 + a^2 / rho^2), see ``potential``).  A corner node is Dirichlet if either adjacent
  side is; its value comes from the bottom/top side when that side is
  Dirichlet, otherwise from the left/right side;
* the surface tangential velocity (section "Velocity Field and Surface
  Tangential Velocity") u_t = (psi_c - psi_b) / d_nc is evaluated on every
  edge whose two end nodes are snapped to the same body and whose length
  exceeds 1e-12 max(hx, hy), in every active cell that has at least one fluid
  node.  psi_c is the mean of the cell's four nodal values, d_nc the
  perpendicular distance from the mean of the four displaced node positions to
  the line through the edge, and the sample angle is the polar angle of the
  edge midpoint about the body centre.  u_t is signed; it tends to
  2 U sin(theta) for a single cylinder.  Samples are ordered by
  (body, cell id, local edge);
* CoPFI = (psi_hi - psi_lo) / (U (y_hi - y_lo)) for the body pair
  (lo, hi).  In the paper's units (U = 2, domain height 0.5, centre distance
  delta * 0.5) this is exactly Q_54 / delta.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import SNAPPED, FLUID, node_coords, spacing, cell_nodes, active_cells
from .fem import assemble

BC_NATURAL, BC_DIRICHLET_UY, BC_DIRICHLET_CYL = 0, 1, 2
BC_DIRICHLET_UX, BC_DIRICHLET_CYLPHI = 3, 4


def dirichlet_mask(grid, flow):
    """Boolean (ny+1, nx+1) mask of Dirichlet nodes."""
    m = np.zeros((grid.ny + 1, grid.nx + 1), dtype=bool)
    L, R, B, T = flow.side_bc
    if L != BC_NATURAL:
        m[:, 0] = True
    if R != BC_NATURAL:
        m[:, -1] = True
    if B != BC_NATURAL:
        m[0, :] = True
    if T != BC_NATURAL:
        m[-1, :] = True
    return m


def _side_value(code, X, Y, flow, circles):
    if code == BC_DIRICHLET_UY:
        return flow.U * Y
    if code == BC_DIRICHLET_CYL:
        cx, cy, a = circles[0]
        dx, dy = X - cx, Y - cy
        rho2 = dx * dx + dy * dy
        return flow.U * dy * (1.0 - a * a / rho2)
    if code == BC_DIRICHLET_UX:
        return flow.U * X
    if code == BC_DIRICHLET_CYLPHI:
        cx, cy, a = circles[0]
        dx, dy = X - cx, Y - cy
        rho2 = dx * dx + dy * dy
        return flow.U * dx * (1.0 + a * a / rho2)
    return np.zeros_like(X)


def dirichlet_values(grid, flow, circles):
    """Full nodal lifting vector g (flat): prescribed values at Dirichlet
    nodes, zero elsewhere."""
    X, Y = node_coords(grid)
    g = np.zeros_like(X)
    L, R, B, T = flow.side_bc
    # vertical sides first, then bottom/top so that they win at corners
    for code, sl in ((L, (slice(None), 0)), (R, (slice(None), -1)),
                     (B, (0, slice(None))), (T, (-1, slice(None)))):
        if code != BC_NATURAL:
            g[sl] = _side_value(code, X[sl], Y[sl], flow, circles)
    return g.ravel()


def dof_numbering(grid, body, flow, nbody):
    """Unknown index of every node: free nodes 0..nfree-1 in node order, body
    b -> nfree + b, Dirichlet -> -1.  Body membership wins over Dirichlet (it
    cannot happen for accepted geometry)."""
    dmask = dirichlet_mask(grid, flow).ravel()
    b = body.ravel().astype(np.int64)
    free = (~dmask) & (b < 0)
    dof = np.full(b.shape, -1, dtype=np.int64)
    nfree = int(free.sum())
    dof[free] = np.arange(nfree)
    isb = b >= 0
    dof[isb] = nfree + b[isb]
    return dof, nfree, nfree + nbody


def selection_matrix(dof, ndof):
    n = dof.size
    rows = np.flatnonzero(dof >= 0)
    return sp.csr_matrix((np.ones(rows.size), (rows, dof[rows])), shape=(n, ndof))


def reduced_system(K, dof, ndof, g):
    """A = T^T K T, b = -T^T K g (see module docstring)."""
    T = selection_matrix(dof, ndof)
    A = (T.T @ K @ T).tocsc()
    b = -(T.T @ (K @ g))
    return A, b, T


@dataclass
class Solution:
    psi: np.ndarray       # flat nodal psi, body nodes carry psi_b
    psi_b: np.ndarray     # (nbody,)
    y: np.ndarray         # reduced unknowns
    A: object
    b: np.ndarray
    T: object
    K: object
    g: np.ndarray
    dof: np.ndarray
    nfree: int
    ndof: int


def solve(mesh, flow, g=None, body_fixed=None):
    """Direct solve of the constrained system for a conformed mesh.

    ``g`` overrides the lifting vector (a full nodal vector whose entries at
    Dirichlet nodes are used).  ``body_fixed`` (a full nodal vector) removes
    the body constraints and prescribes these values at every body node
    instead (used by the patch test)."""
    grid = mesh.grid
    nb = len(mesh.circles)
    K = assemble(mesh)
    if g is None:
        g = dirichlet_values(grid, flow, mesh.circles)
    dmask = dirichlet_mask(grid, flow).ravel()
    body = mesh.body
    if body_fixed is not None:
        isb = body.ravel() >= 0
        g = np.where(isb, np.asarray(body_fixed).ravel(), g)
        dmask = dmask | isb
        body = np.full_like(body, -1)
        nb = 0
    g = np.where(dmask, g, 0.0)
    b_flat = body.ravel().astype(np.int64)
    free = (~dmask) & (b_flat < 0)
    dof = np.full(b_flat.shape, -1, dtype=np.int64)
    nfree = int(free.sum())
    dof[free] = np.arange(nfree)
    dof[b_flat >= 0] = nfree + b_flat[b_flat >= 0]
    ndof = nfree + nb
    A, b, T = reduced_system(K, dof, ndof, g)
    y = spla.splu(A).solve(b) if ndof > 0 else np.zeros(0, dtype=b.dtype)
    psi = g + T @ y
    return Solution(psi, y[nfree:].copy(), y, A, b, T, K, g, dof, nfree, ndof)


def surface_samples(mesh, psi, psi_b):
    """Signed surface tangential velocity samples (see module docstring).

    Returns (theta, u_t, body) arrays ordered by (body, cell id, local edge).
    """
    grid = mesh.grid
    hx, hy = spacing(grid)
    h = max(hx, hy)
    X, Y = mesh.coords()
    Xf, Yf = X.ravel(), Y.ravel()
    kind = mesh.kind.ravel()
    body = mesh.body.ravel().astype(np.int64)
    psi = np.asarray(psi).ravel()
    cn = cell_nodes(grid)
    act = active_cells(grid, mesh.body)
    has_fluid = (kind[cn] == FLUID).any(axis=1)
    cells = np.flatnonzero(act & has_fluid)
    cnc = cn[cells]
    keys_b, keys_c, keys_k, thetas, uts = [], [], [], [], []
    gx = Xf[cnc].mean(axis=1)
    gy = Yf[cnc].mean(axis=1)
    psic = psi[cnc].mean(axis=1)
    for k in range(4):
        a = cnc[:, k]
        c = cnc[:, (k + 1) % 4]
        ok = (kind[a] == SNAPPED) & (kind[c] == SNAPPED) & (body[a] == body[c])
        ex = Xf[c] - Xf[a]
        ey = Yf[c] - Yf[a]
        L = np.hypot(ex, ey)
        ok &= L > 1e-12 * h
        idx = np.flatnonzero(ok)
        bb = body[a[idx]]
        cx = np.array([mesh.circles[q][0] for q in bb], dtype=float)
        cy = np.array([mesh.circles[q][1] for q in bb], dtype=float)
        mx = 0.5 * (Xf[a[idx]] + Xf[c[idx]])
        my = 0.5 * (Yf[a[idx]] + Yf[c[idx]])
        dnc = np.abs(ex[idx] * (gy[idx] - Yf[a[idx]]) - ey[idx] * (gx[idx] - Xf[a[idx]])) / L[idx]
        thetas.append(np.arctan2(my - cy, mx - cx))
        uts.append((psic[idx] - np.asarray(psi_b)[bb]) / dnc)
        keys_b.append(bb)
        keys_c.append(cells[idx])
        keys_k.append(np.full(idx.size, k))
    kb = np.concatenate(keys_b)
    kc = np.concatenate(keys_c)
    kk = np.concatenate(keys_k)
    order = np.lexsort((kk, kc, kb))
    return (np.concatenate(thetas)[order], np.concatenate(uts)[order],
            kb[order].astype(np.int8))


def copfi(psi_b, lo, hi, U, y_lo, y_hi):
    """Q = psi_hi - psi_lo and CoPFI = Q / (U (y_hi - y_lo))."""
    Q = psi_b[hi] - psi_b[lo]
    return Q, Q / (U * (y_hi - y_lo))
