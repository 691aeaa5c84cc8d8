"""Oracle: the velocity-potential solve (flow net companion of psi).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (section "Governing Equation"): for incompressible,
irrotational flow the velocity is also the gradient of a potential phi,
u = grad phi, and phi satisfies the Laplace equation; its contour lines and
those of psi form the flow net.  The discretisation is the one psi uses
(section "Weak formulation"): Q1 elements with K_e = int (grad N)^T (grad N)
over the active cells of the conformed mesh, assembled, solved directly.

Readings (the paper gives no boundary conditions for phi; these are the
potential-flow ones):

* a side with code 3 carries phi = U x (the free stream's potential), code 4
  the isolated-cylinder potential U (x - cx)(1 + a^2 / rho^2) about body 0,
  code 0 is natural (zero normal velocity: the channel walls);
* every body surface is a natural boundary (zero normal velocity through a
  solid body), and no body constraint applies: the body nodes of active
  cells are ordinary unknowns;
* the domain is the union of the active cells (the cells psi uses); nodes in
  no active cell lie inside a body, carry no equation and are reported as NaN;
* corner nodes follow the psi rule (Dirichlet if either side is).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from .fem import assemble
from .mesh import active_cells, cell_nodes
from .solve import dirichlet_mask, dirichlet_values


def in_domain(grid, body):
    """Flat boolean mask of the nodes of at least one active cell."""
    cn = cell_nodes(grid)[active_cells(grid, body)]
    m = np.zeros(grid.nodes, dtype=bool)
    m[cn.ravel()] = True
    return m


@dataclass
class PhiSolution:
    phi: np.ndarray      # flat nodal potential, NaN outside the domain
    free: np.ndarray     # flat mask of the unknowns
    K: object
    g: np.ndarray        # lifting: prescribed values at Dirichlet nodes, else 0
    ndof: int


def phi_solve(mesh, flow):
    """Direct solve of K_ff phi_f = -K_fd g_d over the unknowns f (domain nodes
    that are not Dirichlet) with the Dirichlet values g_d."""
    grid = mesh.grid
    K = assemble(mesh).tocsr()
    dmask = dirichlet_mask(grid, flow).ravel()
    dom = in_domain(grid, mesh.body)
    g = np.where(dmask, dirichlet_values(grid, flow, mesh.circles), 0.0)
    free = dom & ~dmask
    idx = np.flatnonzero(free)
    A = K[idx][:, idx].tocsc()
    b = -(K[idx] @ g)
    phi = g.copy()
    if idx.size:
        phi[idx] = spla.splu(A).solve(b)
    phi[~dom] = np.nan
    return PhiSolution(phi, free, K, g, int(idx.size))


def cell_velocity(mesh, field, kind="phi"):
    """Velocity at the centre of every active cell from a nodal field: grad phi
    (kind="phi") or (psi_y, -psi_x) (kind="psi"), from the bilinear map's
    derivatives at the cell centre.  Returns (cell ids, ux, uy, xc, yc)."""
    grid = mesh.grid
    X, Y = mesh.coords()
    Xf, Yf = X.ravel(), Y.ravel()
    act = np.flatnonzero(active_cells(grid, mesh.body))
    cn = cell_nodes(grid)[act]
    f = np.asarray(field).ravel()[cn]
    x, y = Xf[cn], Yf[cn]
    # node order (i,j), (i+1,j), (i+1,j+1), (i,j+1); derivatives at xi = eta = 0
    dxi = np.array([-1.0, 1.0, 1.0, -1.0]) / 4.0
    deta = np.array([-1.0, -1.0, 1.0, 1.0]) / 4.0
    x_xi, x_eta = x @ dxi, x @ deta
    y_xi, y_eta = y @ dxi, y @ deta
    f_xi, f_eta = f @ dxi, f @ deta
    det = x_xi * y_eta - x_eta * y_xi
    fx = (y_eta * f_xi - y_xi * f_eta) / det
    fy = (-x_eta * f_xi + x_xi * f_eta) / det
    if kind == "phi":
        ux, uy = fx, fy
    else:
        ux, uy = fy, -fx
    return act, ux, uy, x.mean(axis=1), y.mean(axis=1)
