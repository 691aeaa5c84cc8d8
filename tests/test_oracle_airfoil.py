"""Pins of the oracle's sharp-trailing-edge body (Joukowski airfoil) in the mixed-cell
mesh and of the Kutta constraint on it (no GPU).

The inside test (roots of the inverse Joukowski map) is checked against a plain
crossing-number test on 200,000 boundary samples; cut points lie on the boundary (the
level function vanishes there to rounding) and inside their grid edge; the exact
flow vanishes on the boundary and tends to the free stream; linear fields are
reproduced on the airfoil's mixed mesh (patch test).  The Kutta constraint with the
point placed on the exact flow's dividing streamline (the airfoil is shifted so
that the streamline passes through a grid node): the discrete solution of the exact
side data approaches the exact field, psi_b -> 0 and the circulation (summed body
row) -> the Kutta circulation 4 pi U R sin(theta_c - alpha), while the
zero-circulation solve stays an O(1) distance away.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle as O
import workloads as W
from oracle import airfoil as A
from oracle import kutta as KU
from oracle import mixed as M

BASE = A.Joukowski(0.0, 0.0, 0.25, -0.02, 0.02, 0.1)
KPT = (0.75, -0.125)   # a node of every grid on [-4, 4]^2 with n a multiple of 64


def shifted_airfoil():
    """BASE moved vertically so that the Kutta flow's dividing streamline passes
    through KPT."""
    gk = BASE.kutta_circulation(1.0)
    f = lambda y: BASE.psi_exact(np.array([KPT[0]]), np.array([y]), 1.0, gk)[0]
    ystar = brentq(f, -0.2, 0.0, xtol=1e-15)
    return A.Joukowski(0.0, KPT[1] - ystar, 0.25, -0.02, 0.02, 0.1)


def boundary(af, n=200001):
    th = np.linspace(0.0, 2.0 * np.pi, n)
    zr = af.xi0 + af.R * np.cos(th)
    zi = af.eta0 + af.R * np.sin(th)
    d = zr * zr + zi * zi
    xr = zr + af.c ** 2 * zr / d
    xi = zi - af.c ** 2 * zi / d
    ca, sa = af.cs()
    return af.xc + ca * xr + sa * xi, af.yc - sa * xr + ca * xi


def crossing_number(px, py, bx, by):
    inside = np.zeros(px.shape, bool)
    x0, y0 = bx[:-1], by[:-1]
    x1, y1 = bx[1:], by[1:]
    for k in range(px.size):
        cond = (y0 > py[k]) != (y1 > py[k])
        xs = x0[cond] + (py[k] - y0[cond]) * (x1[cond] - x0[cond]) / (y1[cond] - y0[cond])
        inside[k] = np.count_nonzero(xs > px[k]) % 2 == 1
    return inside


def test_inside_test_against_crossing_number():
    af = BASE
    bx, by = boundary(af)
    rng = np.random.default_rng(7)
    px = rng.uniform(-0.6, 0.6, 3000)
    py = rng.uniform(-0.2, 0.2, 3000)
    # keep points at least 1e-3 from the sampled boundary
    d = np.min(np.hypot(px[:, None] - bx[None, ::50], py[:, None] - by[None, ::50]), axis=1)
    keep = d > 1e-3
    ref = crossing_number(px[keep], py[keep], bx, by)
    got = af.contains(px[keep], py[keep])
    assert keep.sum() > 2000 and ref.sum() > 100
    assert np.array_equal(got, ref)


def test_cut_points_on_the_boundary_and_their_edge():
    af = shifted_airfoil()
    g = W.Grid(128, 128, -4.0, 4.0, -4.0, 4.0)
    mm = M.mixed_mesh_bodies(g, [af], 200)
    lv = af.level(mm.pxy[:, 0], mm.pxy[:, 1])
    assert len(mm.pxy) > 20
    assert np.abs(lv).max() <= 1e-15 * af.R2
    X, Y = O.node_coords(g)
    for j, i in zip(*np.nonzero(mm.hpt >= 0)):
        p = mm.pxy[mm.hpt[j, i]]
        assert p[1] == Y[j, i] and X[j, i] <= p[0] <= X[j, i + 1]
    for j, i in zip(*np.nonzero(mm.vpt >= 0)):
        p = mm.pxy[mm.vpt[j, i]]
        assert p[0] == X[j, i] and Y[j, i] <= p[1] <= Y[j + 1, i]


def test_exact_flow_on_the_body_and_far_away():
    af = BASE
    bx, by = boundary(af, 4001)
    for gamma in (0.0, af.kutta_circulation(1.0)):
        assert np.abs(af.psi_exact(bx, by, 1.0, gamma)).max() < 1e-12
    far = af.psi_exact(np.array([300.0, -200.0]), np.array([250.0, -400.0]), 1.0, 0.0)
    np.testing.assert_allclose(far, [250.0, -400.0], rtol=2e-3)


def test_linear_fields_on_the_airfoil_mesh():
    af = shifted_airfoil()
    g = W.Grid(128, 128, -4.0, 4.0, -4.0, 4.0)
    mm = M.mixed_mesh_bodies(g, [af], 200)
    x, y = mm.coords()
    lin = 0.3 + 0.7 * x - 1.3 * y
    flow = W.Flow(1.0, (W.BC_DIRICHLET_UY,) * 4)
    sol = M.mixed_solve(mm, flow, g=lin, body_fixed=lin)
    used = np.zeros(mm.n_nodes, bool)
    used[mm.elem_nodes[mm.elem_nodes >= 0]] = True
    np.testing.assert_allclose(sol.psi[used], lin[used], atol=1e-11)


def test_kutta_point_on_the_dividing_streamline_recovers_the_kutta_flow():
    af = shifted_airfoil()
    gk = af.kutta_circulation(1.0)
    assert af.circulation_through(KPT, 1.0) == pytest.approx(gk, rel=1e-10)
    flow = W.Flow(1.0, (W.BC_DIRICHLET_UY,) * 4)
    errs, pbs, rows, mpc = [], [], [], []
    for n in (64, 128, 256):
        g = W.Grid(n, n, -4.0, 4.0, -4.0, 4.0)
        mm = M.mixed_mesh_bodies(g, [af], 200)
        x, y = mm.coords()
        ex = np.nan_to_num(af.psi_exact(x, y, 1.0, gk))
        s = KU.mixed_solve_kutta(mm, flow, [KPT], g=ex)
        used = np.zeros(mm.n_nodes, bool)
        used[mm.elem_nodes[mm.elem_nodes >= 0]] = True
        errs.append(np.abs(s.psi - ex)[used].max())
        pbs.append(abs(s.psi_b[0]))
        rows.append(s.body_rows[0])
        m = M.mixed_solve(mm, flow, g=ex)
        mpc.append(np.abs(m.psi - ex)[used].max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.3 * errs[0] and errs[2] < 0.015
    assert pbs[0] > pbs[1] > pbs[2] and pbs[2] < 5e-3
    rel = [abs(r - gk) / abs(gk) for r in rows]
    assert rel[0] > rel[1] > rel[2] and rel[2] < 0.02
    assert min(mpc) > 0.2


def test_a_body_the_grid_does_not_resolve_is_rejected():
    """A thin airfoil (0.4% thick) placed between the node rows of a coarse grid holds
    no node: no cut point, no constraint to solve for."""
    g = W.Grid(16, 16, -4.0, 4.0, -4.0, 4.0)
    thin = A.Joukowski(0.0, 0.25, 1.0, -0.001, 0.0, 0.0)
    with pytest.raises(O.GeometryError, match="holds no grid node"):
        M.mixed_mesh_bodies(g, [thin], 10)
