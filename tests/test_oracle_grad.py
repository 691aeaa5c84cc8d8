"""Pins of the oracle's CoPFI derivatives (no GPU).

Three independent routes must agree: complex step through the whole chain,
the discrete adjoint (explicit transposed sweep matrix, per-element complex
step of lambda^T K_e psi, projection Jacobian), and central finite differences
of direct solves.  Symmetry fixes some components exactly: the layout is
mirror-symmetric in y, so dJ/dy of bodies on the axis vanishes, the pair's y
derivatives are opposite, and their x derivatives are equal; moving the pair
apart symmetrically gives dJ/d(delta) = dJ/dy_hi - dJ/dy_lo.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import grad as G


@pytest.fixture(scope="module")
def small_case():
    return W.five_cylinders(96, 48, 0.5, extent=(-6, 6, -3, 3))


@pytest.fixture(scope="module")
def grads(small_case):
    c = small_case
    cs = G.complex_step_gradient(c.grid, c.circles, c.flow, c.pair, 200)
    adj = G.adjoint_gradient(c.grid, c.circles, c.flow, c.pair, 200)
    fd = G.fd_gradient(c.grid, c.circles, c.flow, c.pair, 200)
    return cs, adj, fd


def test_adjoint_equals_complex_step(grads):
    (gc, gd), (ga, gda, _), _ = grads
    scale = np.abs(gc).max()
    np.testing.assert_allclose(ga, gc, rtol=0, atol=1e-10 * scale)
    assert gda == pytest.approx(gd, rel=1e-10)


def test_fd_equals_complex_step(grads):
    (gc, gd), _, (gf, gdf) = grads
    scale = np.abs(gc).max()
    np.testing.assert_allclose(gf, gc, rtol=0, atol=1e-6 * scale)
    assert gdf == pytest.approx(gd, rel=1e-6)


def test_mirror_symmetry_of_gradient(grads):
    (gc, gd), _, _ = grads
    scale = np.abs(gc).max()
    assert np.all(np.abs(gc[:3, 1]) <= 1e-12 * scale)
    assert gc[3, 1] == pytest.approx(-gc[4, 1], rel=1e-10)
    assert gc[3, 0] == pytest.approx(gc[4, 0], rel=1e-8, abs=1e-14 * scale)
    assert gd == pytest.approx(gc[4, 1] - gc[3, 1], rel=1e-10)


def test_sweep_transpose_dot_product():
    c = W.five_cylinders(96, 48, 0.5, extent=(-6, 6, -3, 3))
    k, b = O.classify(c.grid, c.circles)
    rng = np.random.default_rng(7)
    a = rng.normal(size=(2, c.grid.ny + 1, c.grid.nx + 1))
    v = rng.normal(size=c.grid.nodes)
    Sa = O.smooth(c.grid, k, a, 50)[0].ravel()
    MT = G.sweep_matrix(c.grid, k).T.tocsr()
    w = v.copy()
    for _ in range(50):
        w = MT @ w
    assert Sa @ v == pytest.approx(a[0].ravel() @ w, rel=1e-12)


def test_projection_jacobian_matches_complex_step():
    c = W.five_cylinders(96, 48, 0.5, extent=(-6, 6, -3, 3))
    k, b = O.classify(c.grid, c.circles)
    sel, bb, J = G.projection_jacobian(c.grid, c.circles, k, b)
    for body in range(5):
        for comp in range(2):
            cc = [list(map(complex, x)) for x in c.circles]
            cc[body][comp] += 1e-30j
            d = O.snap_displacement(c.grid, [tuple(x) for x in cc], k, b)
            dd = np.imag(np.stack([d[0].ravel()[sel], d[1].ravel()[sel]], 1)) / 1e-30
            mine = np.where((bb == body)[:, None], J[:, :, comp], 0.0)
            np.testing.assert_allclose(dd, mine, atol=1e-14)


def test_radius_derivative_matches_complex_step():
    """conform_grad's radius term against complex step of the projection + sweeps."""
    c = W.five_cylinders(96, 48, 0.5, extent=(-6, 6, -3, 3))
    k, b = O.classify(c.grid, c.circles)
    rng = np.random.default_rng(3)
    gX = rng.normal(size=(2, c.grid.nodes))
    gc, gr = G.conform_grad(c.grid, c.circles, 30, gX, (k, b))
    for body in (0, 4):
        cc = [list(map(complex, x)) for x in c.circles]
        cc[body][2] += 1e-30j
        d0 = O.snap_displacement(c.grid, [tuple(x) for x in cc], k, b)
        d = O.smooth(c.grid, k, d0, 30)
        val = np.imag((d.reshape(2, -1) * gX).sum()) / 1e-30
        assert gr[body] == pytest.approx(val, rel=1e-11)
        for comp in range(2):
            cc = [list(map(complex, x)) for x in c.circles]
            cc[body][comp] += 1e-30j
            d0 = O.snap_displacement(c.grid, [tuple(x) for x in cc], k, b)
            d = O.smooth(c.grid, k, d0, 30)
            val = np.imag((d.reshape(2, -1) * gX).sum()) / 1e-30
            assert gc[body, comp] == pytest.approx(val, rel=1e-11)
