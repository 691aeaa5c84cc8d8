"""GPU parity of the mesh rule and of the matrix-free element apply.

The mesh is compared bit for bit with the oracle (same FP64 operations, no fused
multiply-add).  The apply q = K p is compared element by element with the
oracle's assembled sparse K on seeded N(0,1) vectors: FP64 within 1e-13 of
max|q|, FP32 within 2e-5 of max|q| (float rounding of p, the geometry and ~100
operations per cell).  Sizes span several 64x8 tiles with ragged edges; the
1024x512 five-cylinder mesh runs at full size.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import DEV, need_gpu, say

pytestmark = pytest.mark.gpu

CASES = {
    "cyl64": W.single_cylinder(64),
    "five96x48": W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3)),
    "five_ragged130x67": W.five_cylinders(130, 67, 0.4, extent=(-6.5, 6.5, -3.35, 3.35)),
    "five_gap_lt_h_256x128": W.five_cylinders(256, 128, 0.05),
    "five_1024x512": W.five_cyl_1024(),
    "channel_nobody_70x9": W.Case("channel", W.Grid(70, 9, 0.0, 7.0, 0.0, 0.9), []),
}


@pytest.fixture(scope="module")
def mfp():
    need_gpu()
    import paper_2512_12232_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def meshes(mfp):
    out = {}
    for name, c in CASES.items():
        say(f"[mesh] {name}")
        disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
        torch.cuda.synchronize()
        out[name] = (disp, kind, body, O.conform(c.grid, c.circles, c.nsweeps))
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_mesh_bitwise(meshes, name):
    disp, kind, body, ref = meshes[name]
    assert np.array_equal(kind.cpu().numpy(), ref.kind.ravel())
    assert np.array_equal(body.cpu().numpy(), ref.body.ravel())
    d = disp.cpu().numpy()
    r = ref.disp.reshape(-1)
    bad = np.flatnonzero(d != r)
    assert bad.size == 0, f"{bad.size} displacement entries differ, max {np.abs(d - r).max()}"


def test_mesh_reproducible(mfp):
    c = CASES["five96x48"]
    a = mfp.mesh_conform(c.grid, c.circles, 200, device=DEV)
    b = mfp.mesh_conform(c.grid, c.circles, 200, device=DEV)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_mesh_nsweeps_zero_and_odd(mfp):
    c = CASES["five96x48"]
    for ns in (0, 1, 7):
        disp, kind, body = mfp.mesh_conform(c.grid, c.circles, ns, device=DEV)
        ref = O.conform(c.grid, c.circles, ns)
        assert np.array_equal(disp.cpu().numpy(), ref.disp.reshape(-1)), ns


def test_overlapping_circles_rejected(mfp):
    g = W.Grid(64, 64, -8, 8, -8, 8)
    with pytest.raises(mfp.MfpError) as e:
        mfp.mesh_conform(g, [(0, 0, 1.0), (1.5, 0, 1.0)], 200, device=DEV)
    assert e.value.status == -3


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_apply_matches_assembled_K(meshes, mfp, name, precision):
    disp, kind, body, ref = meshes[name]
    c = CASES[name]
    say(f"[apply] {name} {precision}")
    p = W.random_vector(c.grid.nodes, 1234)
    K = O.assemble(ref)
    qref = K @ p
    q, _ = mfp.element_apply(c.grid, disp, body, torch.from_numpy(p).to(DEV), precision)
    q = q.double().cpu().numpy()
    tol = 1e-13 if precision == "fp64" else 2e-5
    scale = np.abs(qref).max()
    err = np.abs(q - qref).max() / scale
    assert err <= tol, err


def test_apply_symmetric_and_deterministic(meshes, mfp):
    disp, kind, body, ref = meshes["five_gap_lt_h_256x128"]
    c = CASES["five_gap_lt_h_256x128"]
    p = torch.from_numpy(W.random_vector(c.grid.nodes, 1)).to(DEV)
    v = torch.from_numpy(W.random_vector(c.grid.nodes, 2)).to(DEV)
    Ap, _ = mfp.element_apply(c.grid, disp, body, p)
    Av, _ = mfp.element_apply(c.grid, disp, body, v)
    Ap2, _ = mfp.element_apply(c.grid, disp, body, p)
    assert torch.equal(Ap, Ap2)
    a, b = float(v @ Ap), float(p @ Av)
    assert abs(a - b) <= 1e-12 * (abs(a) + 1.0)


def test_apply_constant_and_linear_fields(meshes, mfp):
    """K 1 = 0 and, for a linear field, K u vanishes at every interior node not
    touching an inactive cell (the fast constant-stencil path and the geometric
    path must agree on this)."""
    disp, kind, body, ref = meshes["five_1024x512"]
    c = CASES["five_1024x512"]
    X, Y = ref.coords()
    one = torch.ones(c.grid.nodes, dtype=torch.float64, device=DEV)
    q, _ = mfp.element_apply(c.grid, disp, body, one)
    assert q.abs().max().item() < 1e-12
    lin = torch.from_numpy((0.5 * X + 0.25 * Y).ravel()).to(DEV)
    q, _ = mfp.element_apply(c.grid, disp, body, lin)
    act = O.active_cells(c.grid, ref.body)
    cn = O.cell_nodes(c.grid)
    touched_inactive = np.zeros(c.grid.nodes, bool)
    touched_inactive[cn[~act].ravel()] = True
    interior = np.zeros((c.grid.ny + 1, c.grid.nx + 1), bool)
    interior[1:-1, 1:-1] = True
    sel = interior.ravel() & ~touched_inactive & (ref.body.ravel() < 0)
    assert np.abs(q.cpu().numpy()[sel]).max() < 1e-12
