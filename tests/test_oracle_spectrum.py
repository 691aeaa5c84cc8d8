"""Pins of the oracle's conditioning functions (no GPU).

condition_number: the whole spectrum of the undisplaced operator with Dirichlet
data on all four sides is known in closed form (the assembled 9-point stencil of
the textbook rectangle element is diagonalised by sin(k pi i / nx) sin(l pi j / ny)),
so the dense eigensolver path is checked eigenvalue by eigenvalue and the sparse
(ARPACK) path against the dense one.  lanczos_extremes: on a full Krylov space it
finds the exact extremes; started from a combination of three eigenvectors it
finds exactly those three eigenvalues; from the solve's own right-hand side on a
layout without symmetry its extremes close in on condition_number's from inside.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from oracle.spectrum import condition_number, lanczos_extremes, lanczos_tridiagonal


def rect_closed_form(a, b):
    """Textbook bilinear-rectangle Laplace stiffness, nodes (0,0),(a,0),(a,b),(0,b)."""
    kx = np.array([[2, -2, -1, 1], [-2, 2, 1, -1], [-1, 1, 2, -2], [1, -1, -2, 2]], float)
    ky = np.array([[2, 1, -1, -2], [1, 2, -2, -1], [-1, -2, 2, 1], [-2, -1, 1, 2]], float)
    return b / (6 * a) * kx + a / (6 * b) * ky


def dirichlet_box_system(nx, ny, hx, hy):
    grid = W.Grid(nx, ny, 0.0, nx * hx, 0.0, ny * hy)
    flow = W.Flow(1.0, (W.BC_DIRICHLET_UY,) * 4)
    mesh = O.conform(grid, [], 0)
    return O.solve(mesh, flow)


def symbol_spectrum(nx, ny, hx, hy):
    Ke = rect_closed_form(hx, hy)
    cC, cE, cN, cD = 4 * Ke[0, 0], 2 * Ke[0, 1], 2 * Ke[0, 3], Ke[0, 2]
    th = np.arange(1, nx) * np.pi / nx
    ph = np.arange(1, ny) * np.pi / ny
    ct, cp = np.meshgrid(np.cos(th), np.cos(ph), indexing="ij")
    return np.sort((cC + 2 * cE * ct + 2 * cN * cp + 4 * cD * ct * cp).ravel())


@pytest.mark.parametrize("nx,ny,hx,hy", [(24, 16, 1.0, 1.0), (20, 14, 0.5, 0.25),
                                         (17, 23, 0.1, 0.3)])
def test_dense_spectrum_is_the_stencil_symbol(nx, ny, hx, hy):
    sol = dirichlet_box_system(nx, ny, hx, hy)
    w = np.linalg.eigvalsh(sol.A.toarray())
    ref = symbol_spectrum(nx, ny, hx, hy)
    assert w.size == ref.size
    np.testing.assert_allclose(w, ref, rtol=0, atol=1e-12 * ref.max())
    lmin, lmax, kappa = condition_number(sol.A)
    assert lmin == pytest.approx(ref[0], rel=1e-10)
    assert lmax == pytest.approx(ref[-1], rel=1e-12)
    assert kappa == pytest.approx(ref[-1] / ref[0], rel=1e-10)


def test_sparse_path_matches_dense_path():
    """ARPACK (largest, and shift-invert about 0 for the smallest) on a system above
    the dense limit against the closed form."""
    nx, ny = 90, 60
    sol = dirichlet_box_system(nx, ny, 1.0, 1.0)
    assert sol.A.shape[0] > 4000
    ref = symbol_spectrum(nx, ny, 1.0, 1.0)
    lmin, lmax, _ = condition_number(sol.A)
    assert lmin == pytest.approx(ref[0], rel=1e-8)
    assert lmax == pytest.approx(ref[-1], rel=1e-8)


def test_lanczos_full_space_finds_exact_extremes():
    case = W.single_cylinder(16, half=2.0)
    mesh = O.conform(case.grid, case.circles, 200)
    sol = O.solve(mesh, case.flow)
    A = sol.A.tocsr()
    n = A.shape[0]
    lmin, lmax, _ = condition_number(A)
    b = W.random_vector(n, 7)
    lo, hi = lanczos_extremes(A, b, 3 * n)
    assert lo == pytest.approx(lmin, rel=1e-9)
    assert hi == pytest.approx(lmax, rel=1e-9)


def test_lanczos_from_three_eigenvectors():
    """b in an invariant subspace of dimension 3: three steps give those three
    eigenvalues exactly, whatever the rest of the spectrum."""
    sol = dirichlet_box_system(12, 10, 1.0, 1.0)
    A = sol.A.toarray()
    w, V = np.linalg.eigh(A)
    idx = [4, 30, 77]
    b = V[:, idx] @ np.array([1.0, -0.5, 2.0])
    a, c = lanczos_tridiagonal(sp.csr_matrix(A), b, 3)
    T = np.diag(a) + np.diag(c, 1) + np.diag(c, -1)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(T)), w[idx], rtol=1e-12)
    lo, hi = lanczos_extremes(sp.csr_matrix(A), b, 3)
    assert lo == pytest.approx(w[4], rel=1e-12) and hi == pytest.approx(w[77], rel=1e-12)


def test_lanczos_from_the_right_hand_side_converges_to_the_extremes():
    """CG's own Krylov space (from b = -T^T K g) on a layout without symmetry: the
    Ritz extremes approach lambda_min and lambda_max of A as the steps grow, from
    inside the spectrum (Ritz values interlace)."""
    case = W.five_cylinders_asymmetric(48, 24, (-6, 6, -3, 3))
    mesh = O.conform(case.grid, case.circles, 200)
    sol = O.solve(mesh, case.flow)
    lmin, lmax, _ = condition_number(sol.A)
    A = sol.A.tocsr()
    prev = None
    for m in (10, 40, 160):
        lo, hi = lanczos_extremes(A, sol.b, m)
        assert lmin * (1 - 1e-12) <= lo and hi <= lmax * (1 + 1e-12)
        if prev is not None:
            assert lo <= prev[0] * (1 + 1e-12) and hi >= prev[1] * (1 - 1e-12)
        prev = (lo, hi)
    assert prev[0] == pytest.approx(lmin, rel=1e-6)
    assert prev[1] == pytest.approx(lmax, rel=1e-6)
