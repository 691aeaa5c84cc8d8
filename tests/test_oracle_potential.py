"""Pins of the oracle's velocity-potential solve (no GPU).

Pins: exact reproduction of the free stream phi = U x without bodies, also on a
distorted mesh (isoparametric Q1 patch test, in displaced coordinates); an
independent dense brute-force solve on a tiny mesh with a body; mirror
symmetry (phi even in y for a geometry symmetric about y = 0); the balance of
the Dirichlet reactions (what enters through the inlet leaves through the
outlet); second-order convergence to the isolated-cylinder potential
U x (1 + a^2 / rho^2); and the flow net: the velocity grad phi agrees with the
velocity (psi_y, -psi_x) of the independently pinned stream-function solve.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _phi_mesh_no_body(nx=16, ny=8, disp=None):
    grid = W.Grid(nx, ny, -2.0, 2.0, -1.0, 1.0)
    kind = np.full((ny + 1, nx + 1), O.FLUID, dtype=np.int8)
    body = np.full((ny + 1, nx + 1), -1, dtype=np.int8)
    d = np.zeros((2, ny + 1, nx + 1)) if disp is None else disp
    return O.Mesh(grid, [], kind, body, d)


def test_free_stream_is_exact_without_bodies():
    flow = W.Flow(1.7, (W.BC_DIRICHLET_UX, W.BC_DIRICHLET_UX, W.BC_NATURAL, W.BC_NATURAL))
    mesh = _phi_mesh_no_body()
    sol = O.phi_solve(mesh, flow)
    X, _ = mesh.coords()
    np.testing.assert_allclose(sol.phi, 1.7 * X.ravel(), atol=1e-12)
    assert sol.ndof == (17 - 2) * 9


def test_free_stream_is_exact_on_a_distorted_mesh():
    """Interior nodes moved by up to a quarter cell (boundary nodes fixed): the
    discrete potential is still U times the displaced x coordinate."""
    nx, ny = 16, 8
    rng = np.random.default_rng(3)
    d = np.zeros((2, ny + 1, nx + 1))
    d[:, 1:-1, 1:-1] = rng.uniform(-0.25, 0.25, size=(2, ny - 1, nx - 1)) * (4.0 / nx)
    mesh = _phi_mesh_no_body(nx, ny, d)
    flow = W.Flow(1.0, (W.BC_DIRICHLET_UX, W.BC_DIRICHLET_UX, W.BC_NATURAL, W.BC_NATURAL))
    sol = O.phi_solve(mesh, flow)
    X, _ = mesh.coords()
    np.testing.assert_allclose(sol.phi, X.ravel(), atol=1e-12)


def test_dense_brute_force_with_a_body():
    """Element matrices by 2x2 Gauss written out per cell, a dense global
    matrix, and a dense solve over the domain nodes: the same potential."""
    c = W.potential_flow(W.Case("tiny", W.Grid(16, 8, -4.0, 4.0, -2.0, 2.0),
                                [(0.0, 0.0, 1.0)], W.Flow(1.3)))
    mesh = O.conform(c.grid, c.circles, 200)
    sol = O.phi_solve(mesh, c.flow)
    X, Y = mesh.coords()
    Xf, Yf = X.ravel(), Y.ravel()
    n = c.grid.nodes
    K = np.zeros((n, n))
    g = 1.0 / np.sqrt(3.0)
    pts = [(-g, -g), (g, -g), (g, g), (-g, g)]
    nxp = c.grid.nx + 1
    body = mesh.body.ravel()
    for j in range(c.grid.ny):
        for i in range(c.grid.nx):
            nd = [j * nxp + i, j * nxp + i + 1, (j + 1) * nxp + i + 1, (j + 1) * nxp + i]
            if body[nd[0]] >= 0 and all(body[q] == body[nd[0]] for q in nd):
                continue
            xs, ys = Xf[nd], Yf[nd]
            for xi, eta in pts:
                dN = np.array([[-(1 - eta), (1 - eta), (1 + eta), -(1 + eta)],
                               [-(1 - xi), -(1 + xi), (1 + xi), (1 - xi)]]) / 4.0
                J = dN @ np.stack([xs, ys], axis=1)
                B = np.linalg.solve(J, dN)
                K[np.ix_(nd, nd)] += B.T @ B * np.linalg.det(J)
    dmask = np.zeros(n, dtype=bool)
    dmask[0::nxp] = True
    dmask[nxp - 1::nxp] = True
    dom = np.abs(K).sum(axis=1) > 0
    free = dom & ~dmask
    gv = np.where(dmask, Xf * c.flow.U, 0.0)
    phi = gv.copy()
    phi[free] = np.linalg.solve(K[np.ix_(free, free)], -K[free] @ gv)
    phi[~dom] = np.nan
    np.testing.assert_array_equal(np.isnan(phi), np.isnan(sol.phi))
    np.testing.assert_allclose(phi[dom], sol.phi[dom], rtol=0, atol=1e-12)


def test_mirror_symmetry_and_reaction_balance():
    c = W.potential_flow(W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3)))
    mesh = O.conform(c.grid, c.circles, 200)
    sol = O.phi_solve(mesh, c.flow)
    phi = sol.phi.reshape(c.grid.ny + 1, c.grid.nx + 1)
    np.testing.assert_array_equal(np.isnan(phi), np.isnan(phi[::-1]))
    dom = ~np.isnan(phi)
    np.testing.assert_allclose(phi[dom], phi[::-1][dom], rtol=0, atol=1e-12)
    # K has zero row sums and the free rows vanish: inflow = outflow
    react = sol.K @ np.nan_to_num(sol.phi)
    left = react.reshape(phi.shape)[:, 0].sum()
    right = react.reshape(phi.shape)[:, -1].sum()
    assert abs(left + right) <= 1e-11 * abs(left)
    assert np.abs(react[sol.free]).max() <= 1e-11
    # the bodies slow the flow through the channel: flux below U * height
    assert 0.0 < -left < c.flow.U * 6.0


def test_isolated_cylinder_potential_second_order():
    errs = []
    for n in (32, 64, 128):
        c = W.potential_flow(W.single_cylinder(n, half=4.0), exact_bc=True)
        mesh = O.conform(c.grid, c.circles, 200)
        sol = O.phi_solve(mesh, c.flow)
        X, Y = mesh.coords()
        X, Y = X.ravel(), Y.ravel()
        dom = ~np.isnan(sol.phi)
        ex = X[dom] * (1.0 + 0.25 / (X[dom] ** 2 + Y[dom] ** 2))
        errs.append(np.abs(sol.phi[dom] - ex).max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
    assert errs[2] < 3e-3, errs


def test_flow_net_velocities_agree_with_the_stream_function():
    """grad phi and (psi_y, -psi_x) at cell centres one radius or more off the
    cylinder, both from exact boundary data at 128 x 128 cells, agree with each
    other and with the analytic velocity to O(h^2)."""
    c = W.single_cylinder(128, half=4.0, exact_bc=True)
    cp = W.potential_flow(c, exact_bc=True)
    mesh = O.conform(c.grid, c.circles, 200)
    phi = O.phi_solve(mesh, cp.flow).phi
    psi = O.solve(mesh, c.flow).psi
    _, ux, uy, xc, yc = O.cell_velocity(mesh, np.nan_to_num(phi), "phi")
    _, vx, vy, _, _ = O.cell_velocity(mesh, psi, "psi")
    r2 = xc * xc + yc * yc
    far = r2 > 0.75 ** 2
    a2 = 0.25
    uex = 1.0 - a2 * (xc * xc - yc * yc) / r2 ** 2
    vex = -2.0 * a2 * xc * yc / r2 ** 2
    assert np.hypot(ux - vx, uy - vy)[far].max() < 4e-3
    assert np.hypot(ux - uex, uy - vex)[far].max() < 4e-3
    # orthogonal families: grad phi . grad psi = ux * (-vy) + uy * vx ~ 0
    dot = (ux * -vy + uy * vx)[far] / (np.hypot(ux, uy) * np.hypot(vx, vy))[far]
    assert np.abs(dot).max() < 4e-3
