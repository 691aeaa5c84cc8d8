"""Oracle: derivatives of CoPFI with respect to body centres and the gap ratio.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names shape optimisation and automated sensitivity analysis as the
next step (Conclusions).  The map differentiated here is

    centres c_b  ->  snapped-node displacements d0 (radial projection)
                 ->  d = S d0 (the fixed number of Jacobi sweeps, linear)
                 ->  X = X_bg + d  ->  K(X)  ->  psi_b  ->  CoPFI,

with the node classification frozen (it is piecewise constant in the centres,
so the derivative is that of the frozen-topology map).

Three independent evaluations:

* ``complex_step_gradient``: every parameter perturbed by i*h (h = 1e-30) through
  the whole chain with complex arithmetic and a complex sparse LU; exact to
  rounding, no cancellation;
* ``adjoint_gradient``: one extra solve A lambda = dJ/dy, element shape
  derivatives of lambda^T K_e(X) psi by complex step per coordinate, the
  transposed sweeps S^T built from an explicit sparse sweep matrix, and the
  2x2 projection Jacobian per snapped node;
* ``fd_gradient``: central differences with direct solves, either with the
  classification frozen or rejecting a step that changes it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import (SNAPPED, classify, conform, node_coords, jacobi_weights,
                   update_mask, cell_nodes, active_cells)
from .fem import element_stiffness
from .solve import solve, copfi


def _copfi_value(grid, circles, flow, pair, nsweeps, kind_body):
    mesh = conform(grid, circles, nsweeps, kind_body=kind_body)
    sol = solve(mesh, flow)
    lo, hi = pair
    return copfi(sol.psi_b, lo, hi, flow.U, circles[lo][1], circles[hi][1])[1]


def copfi_value(grid, circles, flow, pair, nsweeps=200):
    kb = classify(grid, circles)
    return float(np.real(_copfi_value(grid, circles, flow, pair, nsweeps, kb)))


def complex_step_gradient(grid, circles, flow, pair, nsweeps=200, h=1e-30,
                          delta_pair=True):
    """dCoPFI/d(cx_b, cy_b) for every body, and dCoPFI/d(delta) where delta
    moves the pair symmetrically (y_hi = +(D + delta), y_lo = -(D + delta)).

    Returns (grad_c of shape (nbody, 2), dJ/ddelta or None)."""
    kb = classify(grid, circles)
    nb = len(circles)
    gc = np.zeros((nb, 2))
    for b in range(nb):
        for k in range(2):
            cc = [list(map(complex, c)) for c in circles]
            cc[b][k] += 1j * h
            J = _copfi_value(grid, [tuple(c) for c in cc], flow, pair, nsweeps, kb)
            gc[b, k] = np.imag(J) / h
    gd = None
    if delta_pair:
        lo, hi = pair
        cc = [list(map(complex, c)) for c in circles]
        cc[hi][1] += 1j * h
        cc[lo][1] -= 1j * h
        J = _copfi_value(grid, [tuple(c) for c in cc], flow, pair, nsweeps, kb)
        gd = np.imag(J) / h
    return gc, gd


def sweep_matrix(grid, kind):
    """One Jacobi sweep as a sparse matrix M on a single displacement
    component: update nodes get wx (E + W) + wy (N + S), others identity."""
    nx1, ny1 = grid.nx + 1, grid.ny + 1
    n = nx1 * ny1
    wx, wy = jacobi_weights(grid)
    upd = update_mask(kind).ravel()
    ids = np.arange(n)
    u = ids[upd]
    fixed = ids[~upd]
    rows = np.concatenate([u, u, u, u, fixed])
    cols = np.concatenate([u + 1, u - 1, u + nx1, u - nx1, fixed])
    vals = np.concatenate([np.full(u.size, wx), np.full(u.size, wx),
                           np.full(u.size, wy), np.full(u.size, wy),
                           np.ones(fixed.size)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def element_shape_gradient(mesh, lam, psi, chunk=1 << 18):
    """gbar[c, n] = d/dX_{n,c} of sum_e lam_e^T K_e(X) psi_e over active cells,
    by complex step in each of the eight coordinates of each cell."""
    grid = mesh.grid
    X, Y = mesh.coords()
    Xf, Yf = np.real(X).ravel(), np.real(Y).ravel()
    act = np.flatnonzero(active_cells(grid, mesh.body))
    cn_all = cell_nodes(grid)
    g = np.zeros((2, grid.nodes))
    h = 1e-30
    for s in range(0, act.size, chunk):
        cn = cn_all[act[s:s + chunk]]
        xe, ye = Xf[cn], Yf[cn]
        le, pe = lam[cn], psi[cn]
        for a in range(4):
            for comp in range(2):
                xc = xe.astype(complex)
                yc = ye.astype(complex)
                if comp == 0:
                    xc[:, a] += 1j * h
                else:
                    yc[:, a] += 1j * h
                K = element_stiffness(xc, yc)
                E = np.einsum("ea,eab,eb->e", le, K, pe)
                np.add.at(g[comp], cn[:, a], np.imag(E) / h)
    return g


def projection_jacobian(grid, circles, kind, body):
    """For each snapped node: d(d0)/d(c_b) = I - (r/rho)(I - u u^T),
    u = (x - c)/rho.  Returns (nodes, body, J) with J of shape (m, 2, 2)."""
    X, Y = node_coords(grid)
    sel = np.flatnonzero(kind.ravel() == SNAPPED)
    bb = body.ravel()[sel].astype(np.int64)
    cx = np.array([circles[b][0] for b in bb])
    cy = np.array([circles[b][1] for b in bb])
    r = np.array([circles[b][2] for b in bb])
    dx = X.ravel()[sel] - cx
    dy = Y.ravel()[sel] - cy
    rho = np.sqrt(dx * dx + dy * dy)
    ux, uy = dx / rho, dy / rho
    f = r / rho
    J = np.empty((sel.size, 2, 2))
    J[:, 0, 0] = 1.0 - f * (1.0 - ux * ux)
    J[:, 0, 1] = f * ux * uy
    J[:, 1, 0] = f * ux * uy
    J[:, 1, 1] = 1.0 - f * (1.0 - uy * uy)
    return sel, bb, J


def conform_grad(grid, circles, nsweeps, gX, kind_body=None):
    """Back-propagate a gradient with respect to the final displacements (shape
    (2, nodes)) through the sweeps and the projection: returns (dL/dc (nbody, 2),
    dL/dr (nbody,)).  Radius: d(d0)/dr = u."""
    kind, body = classify(grid, circles) if kind_body is None else kind_body
    MT = sweep_matrix(grid, kind).T.tocsr()
    gd0 = np.array(gX, dtype=float).reshape(2, -1).copy()
    for _ in range(nsweeps):
        gd0 = np.stack([MT @ gd0[0], MT @ gd0[1]])
    sel, bb, Jp = projection_jacobian(grid, circles, kind, body)
    v = np.stack([gd0[0][sel], gd0[1][sel]], axis=1)
    gc = np.zeros((len(circles), 2))
    np.add.at(gc, bb, np.einsum("mij,mi->mj", Jp, v))
    X, Y = node_coords(grid)
    cx = np.array([circles[b][0] for b in bb])
    cy = np.array([circles[b][1] for b in bb])
    dx = X.ravel()[sel] - cx
    dy = Y.ravel()[sel] - cy
    rho = np.sqrt(dx * dx + dy * dy)
    gr = np.zeros(len(circles))
    np.add.at(gr, bb, (dx * v[:, 0] + dy * v[:, 1]) / rho)
    return gc, gr


def adjoint_gradient(grid, circles, flow, pair, nsweeps=200):
    """Discrete adjoint of the frozen-topology map (see module docstring).

    Returns (grad_c (nbody, 2), dJ/ddelta, extras) where dJ/ddelta uses the
    symmetric pair motion and extras holds intermediate fields."""
    mesh = conform(grid, circles, nsweeps)
    sol = solve(mesh, flow)
    lo, hi = pair
    U = flow.U
    ylo, yhi = circles[lo][1], circles[hi][1]
    Q, J = copfi(sol.psi_b, lo, hi, U, ylo, yhi)
    # dJ/dy: only the two body unknowns of the pair
    rhs = np.zeros(sol.ndof)
    rhs[sol.nfree + hi] = 1.0 / (U * (yhi - ylo))
    rhs[sol.nfree + lo] = -1.0 / (U * (yhi - ylo))
    lam = spla.splu(sol.A).solve(rhs)
    lam_full = sol.T @ lam
    # dJ/dX = -d(lam^T K(X) psi)/dX
    gX = -element_shape_gradient(mesh, lam_full, sol.psi)
    # back through the sweeps and the projection
    gc, _ = conform_grad(grid, circles, nsweeps, gX, (mesh.kind, mesh.body))
    # explicit dependence of CoPFI on y_lo, y_hi
    gc[hi, 1] += -J / (yhi - ylo)
    gc[lo, 1] += J / (yhi - ylo)
    gdelta = gc[hi, 1] - gc[lo, 1]
    return gc, gdelta, dict(J=J, Q=Q, gX=gX, lam=lam_full, sol=sol, mesh=mesh)


def fd_gradient(grid, circles, flow, pair, nsweeps=200, step=1e-5, freeze=True):
    """Central differences with direct solves.

    freeze=True evaluates every perturbed geometry with the unperturbed node
    classification (the frozen-topology map that the gradient describes);
    freeze=False re-classifies and marks an entry NaN when its +-step changes
    the classification (nodes lying exactly on a circle flip for any step)."""
    kb0 = classify(grid, circles)
    nb = len(circles)
    gc = np.full((nb, 2), np.nan)

    def value(cs):
        kb = kb0
        if not freeze:
            kb = classify(grid, cs)
            if not (np.array_equal(kb[0], kb0[0]) and np.array_equal(kb[1], kb0[1])):
                return None
        return float(np.real(_copfi_value(grid, cs, flow, pair, nsweeps, kb)))

    def central(perturb):
        vals = []
        for sgn in (1.0, -1.0):
            cc = [list(c) for c in circles]
            perturb(cc, sgn * step)
            vals.append(value([tuple(c) for c in cc]))
        return np.nan if None in vals else (vals[0] - vals[1]) / (2 * step)

    for b in range(nb):
        for k in range(2):
            def pert(cc, s, b=b, k=k):
                cc[b][k] += s
            gc[b, k] = central(pert)
    lo, hi = pair

    def pert_delta(cc, s):
        cc[hi][1] += s
        cc[lo][1] -= s
    return gc, central(pert_delta)
