"""Pins of the oracle's contour lines (no GPU).

Pins: a linear field on a distorted mesh (its level set is a straight line, and
linear interpolation along straight cell edges is exact): every end point on the
line, the pieces joined end to end, their total length the chord of the line
across the domain; a circle (level set of x^2 + y^2) whose polygon converges to
the circle at second order; a saddle cell written out by hand at two levels
(both pairings); and no segment from a cell inside a body or with a NaN value.
"""
import numpy as np

import oracle as O
import workloads as W


def _mesh(nx, ny, ext, disp=None, body=None):
    grid = W.Grid(nx, ny, *ext)
    kind = np.full((ny + 1, nx + 1), O.FLUID, dtype=np.int8)
    b = np.full((ny + 1, nx + 1), -1, dtype=np.int8) if body is None else body
    d = np.zeros((2, ny + 1, nx + 1)) if disp is None else disp
    return O.Mesh(grid, [], kind, b, d)


def test_linear_field_gives_its_line_exactly():
    nx, ny = 24, 12
    rng = np.random.default_rng(8)
    d = np.zeros((2, ny + 1, nx + 1))
    d[:, 1:-1, 1:-1] = rng.uniform(-0.25, 0.25, size=(2, ny - 1, nx - 1)) * (4.0 / nx)
    mesh = _mesh(nx, ny, (-2.0, 2.0, -1.0, 1.0), d)
    X, Y = mesh.coords()
    f = 0.3 + 0.7 * X - 1.3 * Y
    seg = O.contour(mesh, f, 0.1)
    assert len(seg) > 0
    for k in (0, 2):
        np.testing.assert_allclose(0.3 + 0.7 * seg[:, k] - 1.3 * seg[:, k + 1], 0.1,
                                   rtol=0, atol=1e-12)
    # one polyline: every interior end point is shared by two pieces
    pts = np.concatenate([seg[:, :2], seg[:, 2:]])
    key = np.round(pts / 1e-9).astype(np.int64)
    _, counts = np.unique(key, axis=0, return_counts=True)
    assert (counts == 1).sum() == 2 and set(counts) <= {1, 2}
    # chord of 0.7 x - 1.3 y = -0.2 across [-2, 2] x [-1, 1]: y = (0.7 x + 0.2) / 1.3
    # meets y = -1 at x = -15/7 (outside) and x = -2 at y = -12/13, y = 1 at x = 11/7
    p0 = np.array([-2.0, (0.7 * -2.0 + 0.2) / 1.3])
    p1 = np.array([11.0 / 7.0, 1.0])
    length = np.hypot(seg[:, 2] - seg[:, 0], seg[:, 3] - seg[:, 1]).sum()
    assert abs(length - np.linalg.norm(p1 - p0)) < 1e-12


def test_circle_converges_at_second_order():
    errs = []
    for n in (32, 64, 128):
        mesh = _mesh(n, n, (-1.0, 1.0, -1.0, 1.0))
        X, Y = mesh.coords()
        seg = O.contour(mesh, X * X + Y * Y, 0.25)
        r = np.hypot(seg[:, 0], seg[:, 1])
        length = np.hypot(seg[:, 2] - seg[:, 0], seg[:, 3] - seg[:, 1]).sum()
        errs.append((np.abs(r - 0.5).max(), abs(length - np.pi)))
    for k in range(2):
        assert errs[0][k] / errs[1][k] > 3.0 and errs[1][k] / errs[2][k] > 3.0, errs
    assert errs[2][0] < 1e-4 and errs[2][1] < 1e-3, errs


def test_saddle_cell_both_pairings():
    """Cell (0, 0) of a 2 x 2 mesh on [0, 2] x [0, 2] carries 1, 0, 1, 0 at its nodes
    (0,0), (1,0), (1,1), (0,1); the other nodes are far below every level used."""
    mesh = _mesh(2, 2, (0.0, 2.0, 0.0, 2.0))
    f = np.full((3, 3), -10.0)
    f[0, 0], f[0, 1], f[1, 1], f[1, 0] = 1.0, 0.0, 1.0, 0.0
    seg = O.contour(mesh, f, 0.4)
    own = seg[(seg[:, [0, 2]] <= 1.0).all(axis=1) & (seg[:, [1, 3]] <= 1.0).all(axis=1)]
    # centre 0.5 is above 0.4 like node 0: nodes 1 and 3 are cut off
    np.testing.assert_allclose(own, [[0.6, 0.0, 1.0, 0.4], [0.4, 1.0, 0.0, 0.6]], atol=1e-15)
    seg = O.contour(mesh, f, 0.6)
    own = seg[(seg[:, [0, 2]] <= 1.0).all(axis=1) & (seg[:, [1, 3]] <= 1.0).all(axis=1)]
    # centre 0.5 is below 0.6, node 0 above: nodes 0 and 2 are cut off
    np.testing.assert_allclose(own, [[0.0, 0.4, 0.4, 0.0], [1.0, 0.6, 0.6, 1.0]], atol=1e-15)


def test_inactive_and_nan_cells_give_nothing():
    body = np.full((5, 5), -1, dtype=np.int8)
    body[1:3, 1:3] = 0           # cell (1, 1) has all four nodes in body 0
    mesh = _mesh(4, 4, (0.0, 4.0, 0.0, 4.0), body=body)
    X, Y = mesh.coords()
    f = X.copy()
    seg = O.contour(mesh, f, 1.5)   # the line x = 1.5 crosses cells (1, j), j = 0..3
    assert len(seg) == 3 and not np.any((seg[:, 1] > 1.0) & (seg[:, 1] < 2.0) &
                                        (seg[:, 3] > 1.0) & (seg[:, 3] < 2.0))
    f[3, 1] = np.nan                # node (1, 3): cells (0..1, 2..3) touch it
    seg = O.contour(mesh, f, 1.5)
    assert len(seg) == 1 and np.all(seg[:, [1, 3]] <= 1.0 + 1e-15)
