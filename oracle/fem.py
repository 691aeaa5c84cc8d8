"""Oracle: Q1 element stiffness and its assembly.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Weak formulation": with the Galerkin choice of test functions the
element relation is K_e [psi]_e = f_e with K_e = int_{Omega_e} (grad N)^T
(grad N) dOmega.  Here N are the four bilinear shape functions of a
quadrilateral with nodes in counter-clockwise order, reference coordinates
(xi_a, eta_a) = (-1,-1), (1,-1), (1,1), (-1,1), and the integral is taken with
the 2x2 Gauss rule (points +-1/sqrt(3), unit weights).

Section "Matrix-Free Conjugate Gradient ...": the paper stores element
matrices and never assembles K.  The oracle does the opposite on purpose (it
assembles K as a sparse matrix) so that it shares nothing with the matrix-free
GPU apply; both represent the same operator.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import node_coords, cell_nodes, active_cells

XI_A = np.array([-1.0, 1.0, 1.0, -1.0])
ETA_A = np.array([-1.0, -1.0, 1.0, 1.0])
_G = 1.0 / np.sqrt(3.0)
GAUSS_2X2 = [(-_G, -_G), (_G, -_G), (_G, _G), (-_G, _G)]


def shape_derivatives(xi, eta):
    """dN_a/dxi and dN_a/deta of N_a = (1 + xi_a xi)(1 + eta_a eta)/4."""
    return 0.25 * XI_A * (1.0 + ETA_A * eta), 0.25 * ETA_A * (1.0 + XI_A * xi)


def element_stiffness(xe, ye, return_det=False):
    """K_e for quadrilaterals with node coordinates xe, ye of shape (..., 4).

    At each Gauss point: Jacobian J = [[x_xi, y_xi], [x_eta, y_eta]],
    grad_x N = J^{-1} grad_xi N, contribution det(J) (grad N)^T (grad N).
    Returns K of shape (..., 4, 4) (and the (..., 4) Gauss-point
    determinants when ``return_det``).  Real or complex inputs.
    """
    xe = np.asarray(xe)
    ye = np.asarray(ye)
    K = np.zeros(xe.shape + (4,), dtype=np.result_type(xe, ye, np.float64))
    dets = []
    for (xi, eta) in GAUSS_2X2:
        dxi, deta = shape_derivatives(xi, eta)
        j11 = (dxi * xe).sum(-1)
        j12 = (dxi * ye).sum(-1)
        j21 = (deta * xe).sum(-1)
        j22 = (deta * ye).sum(-1)
        det = j11 * j22 - j12 * j21
        dNdx = (j22[..., None] * dxi - j12[..., None] * deta) / det[..., None]
        dNdy = (-j21[..., None] * dxi + j11[..., None] * deta) / det[..., None]
        K += det[..., None, None] * (dNdx[..., :, None] * dNdx[..., None, :] +
                                     dNdy[..., :, None] * dNdy[..., None, :])
        dets.append(det)
    if return_det:
        return K, np.stack(dets, axis=-1)
    return K


def element_coords(mesh, cells=None):
    """Displaced node coordinates (x, y) of the given cells, shape (nc, 4)."""
    X, Y = mesh.coords()
    cn = cell_nodes(mesh.grid)
    if cells is not None:
        cn = cn[cells]
    return X.ravel()[cn], Y.ravel()[cn]


def assemble(mesh, check_det=True):
    """Assembled global stiffness K (CSR, nodes x nodes) over active cells.

    Raises ValueError if any Gauss-point Jacobian determinant of an active
    cell is not positive (tangled mesh)."""
    act = np.flatnonzero(active_cells(mesh.grid, mesh.body))
    cn = cell_nodes(mesh.grid)[act]
    xe, ye = element_coords(mesh, act)
    Ke, det = element_stiffness(xe, ye, return_det=True)
    if check_det and not np.all(np.real(det) > 0.0):
        raise ValueError("tangled mesh: non-positive Jacobian determinant")
    n = mesh.grid.nodes
    rows = np.repeat(cn, 4, axis=1).ravel()
    cols = np.tile(cn, (1, 4)).ravel()
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    return K


def apply_at_nodes(mesh, p, nodes):
    """(K p)_n for selected nodes n, one node at a time in spirit: for each
    node, the contributions of the (at most four) active cells around it.

    ``p`` is a full nodal vector (flat, length (nx+1)(ny+1)); ``nodes`` are
    flat node ids.  Used to check large-mesh applies on samples without
    assembling K.
    """
    grid = mesh.grid
    nx, ny = grid.nx, grid.ny
    nodes = np.asarray(nodes, dtype=np.int64)
    i = nodes % (nx + 1)
    j = nodes // (nx + 1)
    act = active_cells(grid, mesh.body)
    out = np.zeros(nodes.shape, dtype=np.result_type(p, mesh.disp))
    cn_all = cell_nodes(grid)
    X, Y = mesh.coords()
    Xf, Yf, pf = X.ravel(), Y.ravel(), np.asarray(p).ravel()
    # local index of the node inside each of its four possible cells
    for (ci_off, cj_off, a) in ((-1, -1, 2), (0, -1, 3), (-1, 0, 1), (0, 0, 0)):
        ci = i + ci_off
        cj = j + cj_off
        ok = (ci >= 0) & (ci < nx) & (cj >= 0) & (cj < ny)
        cid = np.where(ok, cj * nx + ci, 0)
        ok &= act[cid]
        cn = cn_all[cid[ok]]
        Ke = element_stiffness(Xf[cn], Yf[cn])
        out[ok] += (Ke[:, a, :] * pf[cn]).sum(-1)
    return out


def rectangle_stiffness(hx, hy):
    """Element stiffness of an undistorted hx x hy rectangle computed by the
    same quadrature (convenience for stencil checks)."""
    xe = np.array([0.0, hx, hx, 0.0])
    ye = np.array([0.0, 0.0, hy, hy])
    return element_stiffness(xe, ye)


__all__ = ["element_stiffness", "element_coords", "assemble", "apply_at_nodes",
           "rectangle_stiffness", "shape_derivatives", "GAUSS_2X2", "node_coords"]
