"""GPU parity of sharp-trailing-edge bodies (Joukowski airfoils) in the mixed-cell mesh
and of the Kutta constraint on it.

Mesh: bit for bit against oracle/mixed.py with oracle/airfoil.py's bodies (the same
FP64 operations without fused multiply-add, cos and sin of the angle of attack from
the C library on both sides): node bodies, cut tables, cut points, displacements,
elements.  Bounding circles as the oracle's.  Solve: the mixed mesh's constrained
solve with the Kutta point behind the trailing edge against the oracle's direct
solve of the nonsymmetric system (psi node by node and psi_b within 1e-9 of max|psi|,
the Kutta equation itself), an airfoil beside a cylinder (zero circulation kept on
the cylinder), FP32 with FP64 refinement, and a 1024 x 512 channel with two airfoils.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle import airfoil as A
from oracle import kutta as KU
from oracle import mixed as M
from gpu_util import DEV, need_gpu, say

pytestmark = pytest.mark.gpu

AF = A.Joukowski(0.0, -0.036879291428751654, 0.25, -0.02, 0.02, 0.1)
AF2 = A.Joukowski(2.1, 0.83, 0.3, -0.03, 0.04, 0.2)
CYL = A.Circle(-2.0, -1.0, 0.5)
UY = W.Flow(1.0, (W.BC_DIRICHLET_UY, W.BC_NATURAL, W.BC_DIRICHLET_UY, W.BC_DIRICHLET_UY))

CASES = {
    "airfoil64": (W.Grid(64, 64, -4.0, 4.0, -4.0, 4.0), [AF], [(0.75, -0.125)]),
    "airfoil256": (W.Grid(256, 256, -4.0, 4.0, -4.0, 4.0), [AF], [(0.75, -0.125)]),
    "airfoil_ragged_190x133": (W.Grid(190, 133, -4.0, 4.0, -2.8, 2.8), [AF], [(0.75, -0.125)]),
    "airfoil_cylinder_two_airfoils": (W.Grid(240, 160, -4.5, 4.5, -3.0, 3.0), [AF, CYL, AF2],
                                      [(0.75, -0.125), None, (2.95, 0.65)]),
}


def as_binding(bd):
    if isinstance(bd, A.Circle):
        return ("circle", bd.cx, bd.cy, bd.r)
    return ("joukowski", bd.xc, bd.yc, bd.c, bd.xi0, bd.eta0, bd.alpha)


@pytest.fixture(scope="module")
def mfp():
    need_gpu()
    import paper_2512_12232_amd as m
    m.load()
    return m


_cache = {}


def pair(mfp, name):
    if name not in _cache:
        g, bodies, _ = CASES[name]
        say(f"[airfoil mesh] {name}")
        gm = mfp.mixed_mesh_bodies(g, [as_binding(b) for b in bodies], 200, device=DEV)
        torch.cuda.synchronize()
        _cache[name] = (gm, M.mixed_mesh_bodies(g, bodies, 200))
    return _cache[name]


def test_bounds_match_the_oracle(mfp):
    got = mfp.body_bounds([as_binding(b) for b in (AF, CYL, AF2)])
    for (cx, cy, r), b in zip(got, (AF, CYL, AF2)):
        ref = b.bounding_circle()
        assert (cx, cy) == (ref[0], ref[1])
        assert r == pytest.approx(ref[2], rel=1e-14)


@pytest.mark.parametrize("name", list(CASES))
def test_mesh_bitwise(mfp, name):
    gm, mm = pair(mfp, name)
    assert np.array_equal(gm.body.cpu().numpy(), mm.body.ravel())
    assert np.array_equal(gm.hpt.cpu().numpy(), mm.hpt.ravel())
    assert np.array_equal(gm.vpt.cpu().numpy(), mm.vpt.ravel())
    pxy = gm.pxy.cpu().numpy()
    assert gm.n_points == len(mm.pxy)
    assert np.array_equal(pxy, mm.pxy), f"max |dP| {np.abs(pxy - mm.pxy).max()}"
    assert np.array_equal(gm.pbody.cpu().numpy(), mm.pbody)
    d = gm.disp.cpu().numpy()
    bad = np.flatnonzero(d != mm.disp.reshape(-1))
    assert bad.size == 0, f"{bad.size} displacement entries differ"
    assert np.array_equal(gm.elem.cpu().numpy(), mm.elem_nodes)
    assert np.array_equal(gm.nne.cpu().numpy(), mm.elem_nne)


def _solve_compare(mfp, name, precision, tol):
    g, bodies, pts = CASES[name]
    gm, mm = pair(mfp, name)
    res = mfp.mixed_psi_solve_kutta(gm, UY, pts, precision=precision, rtol=1e-12)
    assert res.status == mfp.MFP_OK
    ref = KU.mixed_solve_kutta(mm, UY, pts)
    assert res.kutta_nodes == ref.kutta_nodes
    psi = res.psi.cpu().numpy()
    scale = np.abs(ref.psi).max()
    used = np.zeros(mm.n_nodes, bool)
    used[mm.elem_nodes[mm.elem_nodes >= 0]] = True
    err = np.abs(psi - ref.psi)[used].max()
    assert err <= tol * scale, f"max |dpsi| {err:.2e}"
    np.testing.assert_allclose(res.psi_b, ref.psi_b, rtol=0, atol=tol * scale)
    for b, n in enumerate(ref.kutta_nodes):
        if n >= 0:
            assert psi[n] == pytest.approx(res.psi_b[b], abs=tol * scale)
    rows = M.assemble_mixed(mm) @ psi
    N = mm.grid.nodes
    for b, n in enumerate(ref.kutta_nodes):
        rb = rows[N:][mm.pbody == b].sum()
        if n < 0:
            assert abs(rb) <= 1e-8 * scale
        else:
            assert rb == pytest.approx(ref.body_rows[b], rel=1e-6)
    return res


@pytest.mark.parametrize("name", list(CASES))
def test_kutta_solve_matches_oracle(mfp, name):
    _solve_compare(mfp, name, "fp64", 1e-9)


def test_kutta_solve_fp32_refined(mfp):
    _solve_compare(mfp, "airfoil_cylinder_two_airfoils", "fp32_ir", 1e-9)


def test_two_airfoils_full_size_1024x512(mfp):
    """Two airfoils in the 1024 x 512 channel: mesh bit for bit and the Kutta solve
    against the oracle."""
    g = W.Grid(1024, 512, -20.0, 20.0, -10.0, 10.0)
    bodies = [A.Joukowski(-1.0, 0.5, 0.5, -0.04, 0.05, 0.08),
              A.Joukowski(1.5, -0.8, 0.5, -0.04, 0.05, 0.08)]
    gm = mfp.mixed_mesh_bodies(g, [as_binding(b) for b in bodies], 200, device=DEV)
    mm = M.mixed_mesh_bodies(g, bodies, 200)
    assert np.array_equal(gm.pxy.cpu().numpy(), mm.pxy)
    assert np.array_equal(gm.disp.cpu().numpy(), mm.disp.reshape(-1))
    assert np.array_equal(gm.elem.cpu().numpy(), mm.elem_nodes)
    pts = []
    for b in bodies:
        (tx, ty), (dx, dy) = b.trailing_edge()
        pts.append((tx + 0.3 * dx, ty + 0.3 * dy))
    res = mfp.mixed_psi_solve_kutta(gm, UY, pts, rtol=1e-12)
    say(f"[airfoils 1024x512] iters {res.stats['iters']} ms {res.stats['solve_ms']:.1f} "
        f"psi_b {res.psi_b}")
    ref = KU.mixed_solve_kutta(mm, UY, pts)
    scale = np.abs(ref.psi).max()
    np.testing.assert_allclose(res.psi_b, ref.psi_b, rtol=0, atol=1e-8 * scale)
    used = np.zeros(mm.n_nodes, bool)
    used[mm.elem_nodes[mm.elem_nodes >= 0]] = True
    assert np.abs(res.psi.cpu().numpy() - ref.psi)[used].max() <= 1e-8 * scale


def test_unresolved_and_invalid_bodies_rejected(mfp):
    g = W.Grid(16, 16, -4.0, 4.0, -4.0, 4.0)
    with pytest.raises(mfp.MfpError, match="holds no grid node") as e:
        mfp.mixed_mesh_bodies(g, [("joukowski", 0.0, 0.25, 1.0, -0.001, 0.0, 0.0)], 10,
                              device=DEV)
    assert e.value.status == mfp.MFP_E_GEOMETRY
    with pytest.raises(mfp.MfpError) as e:
        mfp.body_bounds([("joukowski", 0.0, 0.0, 1.0, 0.0, 0.1, 0.0)])   # no thickness
    assert e.value.status == mfp.MFP_E_ARG
