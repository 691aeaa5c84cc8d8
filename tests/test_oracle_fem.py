"""Pins of the oracle's Q1 element stiffness and assembly (no GPU).

K_e = int (grad N)^T (grad N) dOmega with the 2x2 Gauss rule (section "Weak
formulation").  The pins do not re-evaluate that formula: they use the
textbook closed form for rectangles, the exact boundary-flux identity for
linear fields on arbitrary quadrilaterals (2x2 Gauss is exact there), and
invariances of the Laplace operator.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def rect_closed_form(a, b):
    """Textbook bilinear-rectangle Laplace stiffness, nodes (0,0),(a,0),(a,b),(0,b)."""
    kx = np.array([[2, -2, -1, 1], [-2, 2, 1, -1], [-1, 1, 2, -2], [1, -1, -2, 2]], float)
    ky = np.array([[2, 1, -1, -2], [1, 2, -2, -1], [-1, -2, 2, 1], [-2, -1, 1, 2]], float)
    return b / (6 * a) * kx + a / (6 * b) * ky


def random_convex_quads(rng, n):
    """Perturbed unit squares (convex, CCW)."""
    base_x = np.array([0.0, 1.0, 1.0, 0.0])
    base_y = np.array([0.0, 0.0, 1.0, 1.0])
    xe = base_x + 0.2 * rng.uniform(-1, 1, (n, 4))
    ye = base_y + 0.2 * rng.uniform(-1, 1, (n, 4))
    s = rng.uniform(0.1, 3.0, (n, 1))
    return s * xe + rng.uniform(-5, 5, (n, 1)), s * ye + rng.uniform(-5, 5, (n, 1))


def test_square_closed_form():
    K = O.element_stiffness(np.array([0.0, 1, 1, 0]), np.array([0.0, 0, 1, 1]))
    ref = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0
    np.testing.assert_allclose(K, ref, atol=1e-15)


@pytest.mark.parametrize("a,b", [(1.0, 1.0), (0.25, 0.1), (2.0, 0.5), (0.0390625, 0.0390625)])
def test_rectangle_closed_form(a, b):
    K = O.element_stiffness(np.array([0.0, a, a, 0]), np.array([0.0, 0, b, b]))
    np.testing.assert_allclose(K, rect_closed_form(a, b), rtol=1e-14, atol=1e-14)


def test_linear_field_boundary_flux_identity():
    """For linear u, (K_e u)_a = 1/2 [gx (y_{a+1} - y_{a-1}) - gy (x_{a+1} - x_{a-1})]
    on any straight-sided quadrilateral (divergence theorem, exact under 2x2 Gauss)."""
    rng = np.random.default_rng(1)
    xe, ye = random_convex_quads(rng, 500)
    K = O.element_stiffness(xe, ye)
    for _ in range(3):
        c0, gx, gy = rng.normal(size=3)
        u = c0 + gx * xe + gy * ye
        lhs = np.einsum("eab,eb->ea", K, u)
        rhs = 0.5 * (gx * (np.roll(ye, -1, 1) - np.roll(ye, 1, 1)) -
                     gy * (np.roll(xe, -1, 1) - np.roll(xe, 1, 1)))
        np.testing.assert_allclose(lhs, rhs, atol=1e-12 * (1 + np.abs(rhs).max()))


def test_symmetry_psd_nullspace():
    rng = np.random.default_rng(2)
    xe, ye = random_convex_quads(rng, 200)
    K = O.element_stiffness(xe, ye)
    np.testing.assert_allclose(K, np.swapaxes(K, 1, 2), atol=1e-13)
    np.testing.assert_allclose(K.sum(-1), 0.0, atol=1e-13)
    ev = np.linalg.eigvalsh(K)
    assert (ev[:, 0] > -1e-12).all()
    assert (ev[:, 1] > 1e-6).all()      # only the constant is in the null space


def test_rigid_motion_scale_and_relabel_invariance():
    rng = np.random.default_rng(3)
    xe, ye = random_convex_quads(rng, 50)
    K = O.element_stiffness(xe, ye)
    th = 0.7
    c, s = np.cos(th), np.sin(th)
    K2 = O.element_stiffness(3.0 * (c * xe - s * ye) + 1.5, 3.0 * (s * xe + c * ye) - 2.0)
    np.testing.assert_allclose(K2, K, atol=1e-12)
    # cyclic relabelling of the nodes permutes rows and columns
    K3 = O.element_stiffness(np.roll(xe, 1, 1), np.roll(ye, 1, 1))
    np.testing.assert_allclose(K3, np.roll(np.roll(K, 1, 1), 1, 2), atol=1e-12)


def undisplaced_mesh(grid):
    kind = np.zeros((grid.ny + 1, grid.nx + 1), np.int8)
    body = np.full_like(kind, -1)
    disp = np.zeros((2,) + kind.shape)
    return O.Mesh(grid, [], kind, body, disp)


@pytest.mark.parametrize("hx,hy", [(1.0, 1.0), (0.5, 0.25)])
def test_assembled_nine_point_stencil(hx, hy):
    g = W.Grid(6, 5, 0.0, 6 * hx, 0.0, 5 * hy)
    K = O.assemble(undisplaced_mesh(g)).toarray()
    nx1 = g.nx + 1
    n = 2 * nx1 + 3
    r, q = hy / hx, hx / hy
    row = K[n]
    assert row[n] == pytest.approx(4.0 / 3.0 * (r + q), abs=1e-14)
    for off in (1, -1):
        assert row[n + off] == pytest.approx(-2.0 / 3.0 * r + q / 3.0, abs=1e-14)
        assert row[n + off * nx1] == pytest.approx(-2.0 / 3.0 * q + r / 3.0, abs=1e-14)
    for off in (nx1 + 1, nx1 - 1, -nx1 + 1, -nx1 - 1):
        assert row[n + off] == pytest.approx(-(r + q) / 6.0, abs=1e-14)
    assert np.count_nonzero(np.abs(row) > 1e-15) == 9


def test_apply_at_nodes_matches_assembled_product():
    case = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    mesh = O.conform(case.grid, case.circles, 200)
    K = O.assemble(mesh)
    p = W.random_vector(case.grid.nodes, 5)
    full = K @ p
    nodes = np.arange(case.grid.nodes)
    np.testing.assert_allclose(O.apply_at_nodes(mesh, p, nodes), full, rtol=1e-13, atol=1e-13)


def test_inactive_cells_are_the_single_body_cells():
    case = W.single_cylinder(64)
    mesh = O.conform(case.grid, case.circles, 200)
    act = O.active_cells(case.grid, mesh.body)
    cn = O.cell_nodes(case.grid)
    b = mesh.body.ravel()[cn]
    for c in range(cn.shape[0]):
        allsame = b[c, 0] >= 0 and (b[c] == b[c, 0]).all()
        assert act[c] == (not allsame)
