"""Pins of the oracle's body-conforming mesh rule (no GPU).

Section "Body-Conforming Grid Generation": just-inside nodes are projected
onto the body, and their displacement is propagated by the Laplace equation
for d (here a fixed number of Jacobi sweeps).  Pins: brute-force pure-Python
classification on small grids, projected points lying on the circle, exact
fixed points of the sweep (linear fields, and x^2 - y^2 which pins the split
of the weights when hx != hy), the finite propagation speed of Jacobi
(graph distance), linearity, mirror symmetry, and an independent sparse-matrix
formulation of the sweep.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import grad as G


def brute_classify(grid, circles):
    hx = (grid.x1 - grid.x0) / grid.nx
    hy = (grid.y1 - grid.y0) / grid.ny
    nx1, ny1 = grid.nx + 1, grid.ny + 1
    body = [[-1] * nx1 for _ in range(ny1)]
    for j in range(ny1):
        for i in range(nx1):
            x = grid.x0 + i * hx
            y = grid.y0 + j * hy
            for b, (cx, cy, r) in enumerate(circles):
                if (x - cx) ** 2 + (y - cy) ** 2 <= r * r:
                    body[j][i] = b
    kind = [[0] * nx1 for _ in range(ny1)]
    for j in range(ny1):
        for i in range(nx1):
            if body[j][i] < 0:
                continue
            near = False
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    jj, ii = j + dj, i + di
                    if 0 <= jj < ny1 and 0 <= ii < nx1 and body[jj][ii] < 0:
                        near = True
            kind[j][i] = O.SNAPPED if near else O.DEEP
    return np.array(kind, np.int8), np.array(body, np.int8)


@pytest.mark.parametrize("case", [
    W.single_cylinder(64),
    W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3)),
    W.five_cylinders(90, 46, 0.05, extent=(-6, 6, -3, 3)),
])
def test_classification_matches_brute_force(case):
    k, b = O.classify(case.grid, case.circles)
    kb, bb = brute_classify(case.grid, case.circles)
    assert np.array_equal(k, kb) and np.array_equal(b, bb)


def test_cylinder_counts_and_nodes_on_circle():
    case = W.single_cylinder(64)
    k, b = O.classify(case.grid, case.circles)
    # 13 body nodes; the 4 nodes exactly on the circle are included (<=)
    assert (b >= 0).sum() == 13
    assert (k == O.SNAPPED).sum() == 12 and (k == O.DEEP).sum() == 1
    d = O.snap_displacement(case.grid, case.circles, k, b)
    X, Y = O.node_coords(case.grid)
    on = np.isclose(X ** 2 + Y ** 2, 0.25, rtol=0, atol=0)
    assert on.sum() == 4
    assert np.all(d[:, on] == 0.0)


def test_projection_lands_on_circle():
    case = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    mesh = O.conform(case.grid, case.circles, 200)
    X, Y = mesh.coords()
    for bi, (cx, cy, r) in enumerate(case.circles):
        sel = (mesh.kind == O.SNAPPED) & (mesh.body == bi)
        rad = np.hypot(X[sel] - cx, Y[sel] - cy)
        np.testing.assert_allclose(rad, r, rtol=4e-16, atol=0)


def test_fixed_nodes_keep_their_displacement():
    case = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    k, b = O.classify(case.grid, case.circles)
    d0 = O.snap_displacement(case.grid, case.circles, k, b)
    d = O.smooth(case.grid, k, d0, 200)
    assert np.array_equal(d[:, k == O.SNAPPED], d0[:, k == O.SNAPPED])
    assert np.all(d[:, k == O.DEEP] == 0)
    for sl in ((slice(None), 0), (slice(None), -1), (0, slice(None)), (-1, slice(None))):
        assert np.all(d[(slice(None),) + sl] == 0)


def _box_kind(grid, border_fixed_ring=True):
    """All nodes fluid; a few interior nodes marked SNAPPED (held fixed)."""
    k = np.zeros((grid.ny + 1, grid.nx + 1), np.int8)
    k[3, 4] = O.SNAPPED
    k[6, 9] = O.SNAPPED
    return k


@pytest.mark.parametrize("hx,hy", [(1.0, 1.0), (1.0, 0.5), (0.3, 0.7)])
def test_sweep_fixed_points_linear_and_harmonic_quadratic(hx, hy):
    g = W.Grid(12, 10, 0.0, 12 * hx, 0.0, 10 * hy)
    k = _box_kind(g)
    X, Y = O.node_coords(g)
    for f in (lambda x, y: 0.3 + 1.7 * x - 0.4 * y, lambda x, y: x * x - y * y + 0.5 * x * y):
        d0 = np.stack([f(X, Y), f(Y, X)])
        d = O.smooth(g, k, d0, 25)
        np.testing.assert_allclose(d, d0, atol=1e-12)
    # a non-harmonic quadratic is not a fixed point
    d0 = np.stack([X * X, Y * Y])
    assert not np.allclose(O.smooth(g, k, d0, 1), d0)


def test_weights_split_matters_for_anisotropic_cells():
    g = W.Grid(12, 10, 0.0, 12.0, 0.0, 5.0)
    wx, wy = O.jacobi_weights(g)
    assert wx == pytest.approx(0.25 / (2 * 1.25)) and wy == pytest.approx(1.0 / (2 * 1.25))
    assert wx + wy == pytest.approx(0.5)


def test_finite_propagation_and_linearity():
    case = W.five_cylinders(160, 80, 0.25, extent=(-10, 10, -5, 5))
    k, b = O.classify(case.grid, case.circles)
    d0 = O.snap_displacement(case.grid, case.circles, k, b)
    ns = 7
    d = O.smooth(case.grid, k, d0, ns)
    # graph distance (4-neighbour) from the snapped set
    dist = np.full(k.shape, 10 ** 6)
    dist[k == O.SNAPPED] = 0
    for _ in range(ns + 2):
        nd = dist.copy()
        nd[1:, :] = np.minimum(nd[1:, :], dist[:-1, :] + 1)
        nd[:-1, :] = np.minimum(nd[:-1, :], dist[1:, :] + 1)
        nd[:, 1:] = np.minimum(nd[:, 1:], dist[:, :-1] + 1)
        nd[:, :-1] = np.minimum(nd[:, :-1], dist[:, 1:] + 1)
        dist = nd
    far = dist > ns
    assert np.all(d[:, far] == 0.0)
    assert np.any(d[:, (dist == ns) & (k == O.FLUID)] != 0.0)
    # superposition of two snapped data sets
    rng = np.random.default_rng(0)
    snap = k == O.SNAPPED
    a = np.where(snap, rng.normal(size=d0.shape), 0.0)
    c = np.where(snap, rng.normal(size=d0.shape), 0.0)
    np.testing.assert_allclose(O.smooth(case.grid, k, a + c, 30),
                               O.smooth(case.grid, k, a, 30) + O.smooth(case.grid, k, c, 30),
                               atol=1e-13)


def test_sweep_equals_sparse_matrix_power():
    case = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    k, b = O.classify(case.grid, case.circles)
    d0 = O.snap_displacement(case.grid, case.circles, k, b)
    M = G.sweep_matrix(case.grid, k)
    v = d0[0].ravel().copy()
    for _ in range(40):
        v = M @ v
    np.testing.assert_allclose(O.smooth(case.grid, k, d0, 40)[0].ravel(), v, atol=1e-15)


def test_mirror_symmetric_mesh_is_bitwise_mirrored():
    case = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    mesh = O.conform(case.grid, case.circles, 200)
    assert np.array_equal(mesh.kind, mesh.kind[::-1])
    assert np.array_equal(mesh.disp[0], mesh.disp[0][::-1])
    assert np.array_equal(mesh.disp[1], -mesh.disp[1][::-1])


@pytest.mark.parametrize("case", [
    W.single_cylinder(64),
    W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3)),
    W.five_cylinders(256, 128, 0.05),
    W.five_cylinders(256, 128, 2.0),
])
def test_active_cells_untangled(case):
    mesh = O.conform(case.grid, case.circles, 200)
    act = np.flatnonzero(O.active_cells(case.grid, mesh.body))
    xe, ye = O.element_coords(mesh, act)
    _, det = O.element_stiffness(xe, ye, return_det=True)
    hx, hy = O.spacing(case.grid)
    # 1/4 of the cell area is det J of an undistorted cell
    assert det.min() / (0.25 * hx * hy) > 0.05


@pytest.mark.parametrize("circles,msg", [
    ([(0.0, 0.0, 1.0), (1.5, 0.0, 1.0)], "overlap"),
    ([(0.0, 0.0, 0.3)], "radius"),
    ([(7.4, 0.0, 0.5)], "boundary"),
    ([(0.0, -7.6, 0.5)], "boundary"),
])
def test_geometry_rejected(circles, msg):
    g = W.Grid(64, 64, -8, 8, -8, 8)
    with pytest.raises(O.GeometryError, match=msg):
        O.check_geometry(g, circles)
