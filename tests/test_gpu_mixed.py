"""GPU parity of the mixed-cell mesh, its element product and its constrained solve.

Mesh: the library's cut points, node displacements, tags and elements are compared
bit for bit with the oracle's (the same FP64 operations without fused multiply-add;
integer tables exactly).  Apply: q = K p against the oracle's assembled sparse
matrix on seeded N(0,1) vectors, each entry within 2.5e-13 of the sum over its
elements of max|K_e| sum_b |p_b| (the element matrices differ only by rounding,
which for a Gauss-integrated distorted quadrilateral reaches about 6e-14 of
max|K_e| on either side).  Solve: CG to
1e-12 against the oracle's direct solve; the FP64 residual of the GPU's unknowns,
recomputed on the CPU with the oracle's reduced matrix, must be within 1e-11 of
||b||, and the error of the unknowns within ||r|| / lambda_min (lambda_min of the
oracle's reduced matrix by shift-invert Lanczos) plus 1e-12 of their size for the
direct solve's own rounding.  Sizes run from one cylinder on 32 x 32 cells to the
1024 x 512 five-cylinder channel at full size, with a ragged grid and a cell cut
into a pentagon among them; geometries the mesh rejects return MFP_E_GEOMETRY.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle as O
import workloads as W
from oracle import mixed as M
from gpu_util import DEV, need_gpu, say

pytestmark = pytest.mark.gpu

CASES = {
    "cyl32": W.single_cylinder(32, half=4.0),
    "five96x48": W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3)),
    "five_asym120x60": W.five_cylinders_asymmetric(120, 60, extent=(-6, 6, -3, 3)),
    "five_ragged130x67": W.five_cylinders(130, 67, 0.4, extent=(-6.5, 6.5, -3.35, 3.35)),
    "pentagon12": W.Case("pentagon", W.Grid(12, 12, -4.0, 8.0, -4.0, 8.0), [(1.7, 1.7, 2.0)],
                         W.Flow(1.0, (W.BC_DIRICHLET_UY,) * 4), nsweeps=0),
    "five_1024x512": W.five_cyl_1024(),
}
SMALL = [k for k in CASES if k != "five_1024x512"]


@pytest.fixture(scope="module")
def mfp():
    need_gpu()
    import paper_2512_12232_amd as m
    m.load()
    return m


_cache = {}


def pair(mfp, name):
    """(GPU mesh, oracle mesh) of a case, built once."""
    if name not in _cache:
        c = CASES[name]
        say(f"[mixed mesh] {name}")
        gm = mfp.mixed_mesh(c.grid, c.circles, c.nsweeps, device=DEV)
        torch.cuda.synchronize()
        _cache[name] = (gm, M.mixed_mesh(c.grid, c.circles, c.nsweeps))
    return _cache[name]


def oracle_pedge(mm):
    g = mm.grid
    nh = (g.ny + 1) * g.nx
    pe = np.zeros(len(mm.pxy), dtype=np.int64)
    js, is_ = np.nonzero(mm.hpt >= 0)
    pe[mm.hpt[js, is_]] = js * g.nx + is_
    js, is_ = np.nonzero(mm.vpt >= 0)
    pe[mm.vpt[js, is_]] = nh + js * (g.nx + 1) + is_
    return pe


@pytest.mark.parametrize("name", list(CASES))
def test_mesh_bitwise(mfp, name):
    gm, mm = pair(mfp, name)
    g = mm.grid
    assert np.array_equal(gm.body.cpu().numpy(), mm.body.ravel())
    assert np.array_equal(gm.hpt.cpu().numpy(), mm.hpt.ravel())
    assert np.array_equal(gm.vpt.cpu().numpy(), mm.vpt.ravel())
    assert gm.n_points == len(mm.pxy)
    pxy = gm.pxy.cpu().numpy()
    assert np.array_equal(pxy, mm.pxy), f"max |dP| {np.abs(pxy - mm.pxy).max()}"
    assert np.array_equal(gm.pbody.cpu().numpy(), mm.pbody)
    assert np.array_equal(gm.pedge.cpu().numpy(), oracle_pedge(mm))
    d = gm.disp.cpu().numpy()
    r = mm.disp.reshape(-1)
    bad = np.flatnonzero(d != r)
    assert bad.size == 0, f"{bad.size} displacement entries differ, max {np.abs(d - r).max()}"
    assert gm.n_elems == len(mm.elem_nne)
    assert np.array_equal(gm.elem.cpu().numpy(), mm.elem_nodes)
    assert np.array_equal(gm.nne.cpu().numpy(), mm.elem_nne)
    assert gm.n_tri == int((mm.elem_nne == 3).sum())
    first = np.concatenate([[0], np.cumsum(np.bincount(mm.elem_cell, minlength=g.nx * g.ny))])
    assert np.array_equal(gm.cell_first.cpu().numpy(), first)


def test_pentagon_cell_split(mfp):
    gm, mm = pair(mfp, "pentagon12")
    cid = 7 * 12 + 7
    f = gm.cell_first.cpu().numpy()
    assert f[cid + 1] - f[cid] == 2
    assert list(gm.nne.cpu().numpy()[f[cid]:f[cid + 1]]) == [3, 4]


def element_scale(mm, Ke, p):
    """Per node: sum over its elements e of max|K_e| * sum_b |p_b|.  A Gauss-integrated
    K_e of a distorted quadrilateral carries FP64 rounding of up to about 6e-14 of
    max|K_e| (against extended precision, on the 1024 x 512 mixed mesh): the bar of
    the apply is a few times that on either side."""
    me = np.abs(Ke).max(axis=(1, 2))
    en = mm.elem_nodes
    pa = np.where(en >= 0, np.abs(p)[np.maximum(en, 0)], 0.0).sum(axis=1)
    out = np.zeros(mm.n_nodes)
    for a in range(4):
        ok = en[:, a] >= 0
        np.add.at(out, en[ok, a], (me * pa)[ok])
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_apply_matches_assembled(mfp, name):
    gm, mm = pair(mfp, name)
    A = M.assemble_mixed(mm)
    Ke = M.element_matrices(mm)
    for seed in (0, 1):
        p = W.random_vector(mm.n_nodes, 70 + seed)
        q, ms = mfp.mixed_element_apply(gm, torch.from_numpy(p).to(DEV))
        q = q.cpu().numpy()
        ref = A @ p
        scale = element_scale(mm, Ke, p)
        err = np.abs(q - ref)
        assert np.all(err <= 2.5e-13 * scale + 1e-300), \
            f"worst {np.max(err / np.maximum(scale, 1e-300)):.2e} of the element scale"
        assert ms > 0.0


def test_apply_deterministic(mfp):
    gm, mm = pair(mfp, "five_ragged130x67")
    p = torch.from_numpy(W.random_vector(mm.n_nodes, 5)).to(DEV)
    q1, _ = mfp.mixed_element_apply(gm, p)
    q2, _ = mfp.mixed_element_apply(gm, p, repeat=3)
    assert torch.equal(q1, q2)


_sol = {}


def oracle_solution(mm, flow, name):
    if name not in _sol:
        say(f"[mixed oracle solve] {name}")
        _sol[name] = M.mixed_solve(mm, flow)
    return _sol[name]


@pytest.mark.parametrize("name", SMALL)
def test_solve_matches_direct(mfp, name):
    c = CASES[name]
    gm, mm = pair(mfp, name)
    ref = oracle_solution(mm, c.flow, name)
    res = mfp.mixed_psi_solve(gm, c.flow, rtol=1e-12, pair=c.pair)
    assert res.status == mfp.MFP_OK
    psi = res.psi.cpu().numpy()
    # the GPU's unknowns in the oracle's numbering, and their FP64 residual on the CPU
    y = np.zeros(ref.ndof)
    free = ref.dof[:mm.grid.nodes] >= 0
    y[ref.dof[:mm.grid.nodes][free]] = psi[:mm.grid.nodes][free]
    y[ref.nfree:] = res.psi_b
    r = ref.b - ref.A @ y
    bn = np.linalg.norm(ref.b)
    assert np.linalg.norm(r) <= 1e-11 * bn, f"relres {np.linalg.norm(r) / bn:.2e}"
    assert res.stats["relres_true"] <= 1e-11
    lmin = spla.eigsh(ref.A, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
    ysol = spla.spsolve(ref.A, ref.b)
    bound = np.linalg.norm(r) / lmin + 1e-12 * np.abs(ysol).max()
    err = np.linalg.norm(y - ysol)
    assert err <= bound, f"|y - y*| {err:.2e} > {bound:.2e}"
    # psi: Dirichlet values exact, unused nodes 0, cut points psi_b
    used = np.zeros(mm.n_nodes, bool)
    used[mm.elem_nodes[mm.elem_nodes >= 0]] = True
    dm = np.concatenate([O.dirichlet_mask(mm.grid, c.flow).ravel() & (mm.body.ravel() < 0),
                         np.zeros(len(mm.pxy), bool)])
    # the same expression, possibly with a fused multiply-add: within a few ulp
    np.testing.assert_allclose(psi[dm], ref.psi[dm], rtol=0,
                               atol=1e-14 * max(1.0, np.abs(ref.psi).max()))
    assert np.all(psi[:mm.grid.nodes][mm.body.ravel() >= 0] == 0.0)
    np.testing.assert_array_equal(psi[mm.grid.nodes:], np.asarray(res.psi_b)[mm.pbody])
    assert res.stats["n_free"] == ref.nfree and res.stats["n_dof"] == ref.ndof
    np.testing.assert_allclose(psi[used], ref.psi[used], rtol=0,
                               atol=bound + 1e-12 * np.abs(ref.psi).max())


@pytest.mark.parametrize("name", ["five96x48", "five_asym120x60"])
def test_solve_fp32_refined(mfp, name):
    """FP32 iterations with FP64 residual replacement reach the FP64 solve's accuracy."""
    c = CASES[name]
    gm, mm = pair(mfp, name)
    ref = oracle_solution(mm, c.flow, name)
    res = mfp.mixed_psi_solve(gm, c.flow, precision="fp32_ir", rtol=1e-12, pair=c.pair)
    assert res.status == mfp.MFP_OK
    assert res.stats["relres_true"] <= 1e-11
    lmin = spla.eigsh(ref.A, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
    bound = 1e-11 * np.linalg.norm(ref.b) / lmin + 1e-12 * np.abs(ref.psi).max()
    np.testing.assert_allclose(res.psi_b, ref.psi_b, rtol=0, atol=bound)


def test_solve_full_size_1024x512(mfp):
    c = CASES["five_1024x512"]
    gm, mm = pair(mfp, "five_1024x512")
    ref = oracle_solution(mm, c.flow, "five_1024x512")
    res = mfp.mixed_psi_solve(gm, c.flow, rtol=1e-12, pair=c.pair)
    say(f"[mixed solve 1024x512] iters {res.stats['iters']} ms {res.stats['solve_ms']:.1f}")
    assert res.status == mfp.MFP_OK
    psi = res.psi.cpu().numpy()
    y = np.zeros(ref.ndof)
    free = ref.dof[:mm.grid.nodes] >= 0
    y[ref.dof[:mm.grid.nodes][free]] = psi[:mm.grid.nodes][free]
    y[ref.nfree:] = res.psi_b
    r = ref.b - ref.A @ y
    bn = np.linalg.norm(ref.b)
    assert np.linalg.norm(r) <= 1e-11 * bn, f"relres {np.linalg.norm(r) / bn:.2e}"
    # a-posteriori bound |y - y*|_2 <= |r|_2 / lambda_min (lambda_min about 4.0e-5,
    # kappa about 2.7e6), plus the direct solve's own rounding
    lmin = spla.eigsh(ref.A, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
    bound = np.linalg.norm(r) / lmin + 1e-12 * np.abs(ref.psi).max()
    say(f"[mixed 1024x512] lambda_min {lmin:.3e} bound {bound:.2e} "
        f"psi_b err {np.abs(np.asarray(res.psi_b) - ref.psi_b).max():.2e}")
    np.testing.assert_allclose(res.psi_b, ref.psi_b, rtol=0, atol=bound)
    used = np.zeros(mm.n_nodes, bool)
    used[mm.elem_nodes[mm.elem_nodes >= 0]] = True
    np.testing.assert_allclose(psi[used], ref.psi[used], rtol=0, atol=bound)
    dy = c.flow.U * (c.circles[c.pair[1]][1] - c.circles[c.pair[0]][1])
    assert abs(res.copfi - (ref.psi_b[c.pair[1]] - ref.psi_b[c.pair[0]]) / dy) <= 2 * bound / dy


def test_geometry_rejected(mfp):
    g = W.Grid(40, 20, -5, 5, -2.5, 2.5)
    # two disjoint circles holding the neighbouring nodes (-0.25, 0) and (0, 0)
    c = [(-1.04, 0.0, 0.8), (0.78, 0.0, 0.8)]
    assert mfp.check_geometry(g, c) == mfp.MFP_OK
    with pytest.raises(mfp.MfpError, match="two bodies"):
        mfp.mixed_mesh(g, c, 10, device=DEV)


def test_no_body_channel(mfp):
    """No body: every cell a quadrilateral and psi = U y reproduced (Q1 elements hold
    linear fields): the lifting's residual is rounding (about 1e-15), which the solve
    returns amplified by at most 1/lambda_min (about 10 here)."""
    g = W.Grid(70, 9, 0.0, 7.0, 0.0, 0.9)
    flow = W.Flow(1.0, (W.BC_DIRICHLET_UY,) * 4)
    gm = mfp.mixed_mesh(g, [], 200, device=DEV)
    assert gm.n_points == 0 and gm.n_elems == 70 * 9 and gm.n_tri == 0
    res = mfp.mixed_psi_solve(gm, flow, rtol=1e-12)
    assert res.status == mfp.MFP_OK
    y = np.repeat(np.linspace(0.0, 0.9, 10), 71)
    np.testing.assert_allclose(res.psi.cpu().numpy(), y, rtol=0, atol=1e-11)
