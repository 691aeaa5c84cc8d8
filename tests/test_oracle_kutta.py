"""Pins of the oracle's Kutta constraint (no GPU).

The constraint psi(K_b) = psi_b in place of a body's zero-circulation row
(section "Boundary Conditions", trailing-edge paragraph) is pinned by the exact
lifting cylinder: uniform flow past a circle with circulation Gamma has
psi = U y (1 - a^2/r^2) - Gamma/(2 pi) ln(r/a), zero on the circle, and choosing
Gamma so that the zero streamline passes through a grid node K makes K a valid
Kutta point.  With that field's values on the box, the solve with the Kutta row
converges at second order to it (psi_b -> 0, the summed body row -> Gamma), while
the zero-circulation solve of the same data stays an O(1) distance away.  Also: a
dense system written out by hand on a tiny mesh, a Kutta point on the symmetry
axis of a non-lifting layout (the zero-circulation solution already satisfies
it), a mixed case where the other body's row stays zero, and the node rule.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import kutta as KU

POINT = (0.875, -0.375)   # a node of the 64, 128 and 256 grids on [-4, 4]^2


def _lifting_case(n):
    c = W.single_cylinder(n, half=4.0)
    mesh = O.conform(c.grid, c.circles, 200)
    X, Y = O.node_coords(c.grid)
    gamma = KU.circulation_through(POINT, 1.0, (0.0, 0.0), 0.5)
    g = KU.lifting_cylinder_psi(X, Y, 1.0, (0.0, 0.0), 0.5, gamma).ravel()
    flow = W.Flow(1.0, (W.BC_DIRICHLET_UY,) * 4)
    Xd = (X + mesh.disp[0]).ravel()
    Yd = (Y + mesh.disp[1]).ravel()
    exact = KU.lifting_cylinder_psi(Xd, Yd, 1.0, (0.0, 0.0), 0.5, gamma)
    return mesh, flow, g, exact, gamma


def test_lifting_cylinder_converges_with_the_kutta_row():
    errs, pbs, rows, mpc = [], [], [], []
    for n in (64, 128, 256):
        mesh, flow, g, exact, gamma = _lifting_case(n)
        fluid = mesh.body.ravel() < 0
        s = KU.solve_kutta(mesh, flow, [POINT], g=g)
        errs.append(np.abs(s.psi - exact)[fluid].max())
        pbs.append(abs(s.psi_b[0]))
        rows.append(s.body_rows[0])
        m = O.solve(mesh, flow, g=g)
        mpc.append(np.abs(m.psi - exact)[fluid].max())
    assert errs[0] > errs[1] > errs[2] and errs[1] / errs[2] > 3.0 and errs[2] < 1e-3
    assert pbs[0] > pbs[1] > pbs[2] and pbs[2] < 5e-4
    # the summed body row is the circulation around the body
    rel = [abs(r - gamma) / abs(gamma) for r in rows]
    assert rel[0] > rel[1] > rel[2] and rel[2] < 2e-3
    # zero circulation cannot meet these data
    assert min(mpc) > 0.5


def test_dense_system_written_out():
    case = W.single_cylinder(12, half=1.5)
    mesh = O.conform(case.grid, case.circles, 200)
    pt = (0.875, -0.375)
    s = KU.solve_kutta(mesh, case.flow, [pt])
    K = O.assemble(mesh).toarray()
    n = K.shape[0]
    body = mesh.body.ravel()
    dmask = O.dirichlet_mask(case.grid, case.flow).ravel()
    g = np.where(dmask, O.dirichlet_values(case.grid, case.flow, case.circles), 0.0)
    unknown = [k for k in range(n) if not dmask[k] and body[k] < 0]
    idx = {k: q for q, k in enumerate(unknown)}
    m = len(unknown) + 1
    M = np.zeros((m, m))
    rhs = np.zeros(m)
    for k in unknown:
        for l in range(n):
            if K[k, l] == 0.0:
                continue
            if l in idx:
                M[idx[k], idx[l]] += K[k, l]
            elif body[l] >= 0:
                M[idx[k], m - 1] += K[k, l]
            else:
                rhs[idx[k]] -= K[k, l] * g[l]
    kn = KU.kutta_node(case.grid, pt)
    M[m - 1, idx[kn]] = 1.0
    M[m - 1, m - 1] = -1.0
    y = np.linalg.solve(M, rhs)
    np.testing.assert_allclose(s.psi_b[0], y[-1], atol=1e-12)
    np.testing.assert_allclose(s.psi[unknown], y[:-1], atol=1e-12)
    assert s.psi[kn] == pytest.approx(s.psi_b[0], abs=1e-13)


def test_point_on_the_axis_of_a_symmetric_layout_changes_nothing():
    case = W.single_cylinder(64, half=4.0)
    mesh = O.conform(case.grid, case.circles, 200)
    s = KU.solve_kutta(mesh, case.flow, [(1.0, 0.0)])
    m = O.solve(mesh, case.flow)
    np.testing.assert_allclose(s.psi, m.psi, atol=1e-11)
    assert abs(s.body_rows[0]) < 1e-10


def test_other_bodies_keep_zero_circulation():
    case = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    mesh = O.conform(case.grid, case.circles, 200)
    pts = [None, None, None, (0.75, -1.5), None]   # behind the lower transverse body
    s = KU.solve_kutta(mesh, case.flow, pts)
    for b in (0, 1, 2, 4):
        assert abs(s.body_rows[b]) < 1e-10
    kn = s.kutta_nodes[3]
    assert s.psi[kn] == pytest.approx(s.psi_b[3], abs=1e-12)
    assert abs(s.body_rows[3]) > 1e-3     # body 3 now carries circulation


def test_node_rule_and_rejections():
    g = W.Grid(8, 8, 0.0, 8.0, 0.0, 8.0)
    assert KU.kutta_node(g, (2.5, 3.49)) == 3 * 9 + 3   # ties to the larger index
    assert KU.kutta_node(g, (2.49, 3.51)) == 4 * 9 + 2
    with pytest.raises(KU.KuttaError):
        KU.kutta_node(g, (9.0, 1.0))
    case = W.single_cylinder(32, half=4.0)
    mesh = O.conform(case.grid, case.circles, 200)
    with pytest.raises(KU.KuttaError):
        KU.solve_kutta(mesh, case.flow, [(0.0, 0.0)])      # inside the body
    with pytest.raises(KU.KuttaError):
        KU.solve_kutta(mesh, case.flow, [(-4.0, 1.0)])     # on the Dirichlet inlet
