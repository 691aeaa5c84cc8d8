"""GPU adjoint (psi_grad + mesh_conform_grad + the autograd Function) against the
oracle: the shape term against the oracle's per-element complex-step derivative,
the mesh back-propagation against the oracle's transposed sweep matrix, and the
full CoPFI gradient against complex step through the whole oracle pipeline (the
frozen-topology derivative) within 1e-7 of max|grad| (the stated bar is 1e-6
relative to finite differences).  At the full 2048x1024 size: the oracle's
discrete-adjoint gradient stored in tests/golden, the mirror-symmetry identities
and central finite differences of warm-started GPU solves.
"""
import os

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle import grad as G
from gpu_util import DEV, need_gpu, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))

SMALL = W.five_cylinders(96, 48, 0.5, extent=(-6, 6, -3, 3))
SMALL_GAP = W.five_cylinders(130, 67, 0.1, extent=(-6.5, 6.5, -3.35, 3.35))


@pytest.fixture(scope="module")
def mfp():
    need_gpu()
    import paper_2512_12232_amd as m
    m.load()
    return m


def gpu_forward(mfp, c, rtol=1e-13):
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    res = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=rtol, pair=c.pair)
    return disp, kind, body, res


@pytest.mark.parametrize("c", [SMALL, SMALL_GAP], ids=["five96", "five130_gap0.1"])
def test_shape_term_matches_oracle(mfp, c):
    say(f"[adjoint shape] {c.name}")
    disp, kind, body, res = gpu_forward(mfp, c)
    gX, explicit, stats, status, _ = mfp.psi_grad(c.grid, c.circles, disp, kind, body, c.flow,
                                               res.psi, res.psi_b, dL_dcopfi=1.0,
                                               pair=c.pair, rtol=1e-13)
    assert status == 0
    _, _, ex = G.adjoint_gradient(c.grid, c.circles, c.flow, c.pair, c.nsweeps)
    ref = ex["gX"].reshape(-1)
    got = gX.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()


def test_mesh_backprop_matches_oracle(mfp):
    c = SMALL
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, 200, device=DEV)
    g = W.random_vector(2 * c.grid.nodes, 99)
    dcen, drad = mfp.mesh_conform_grad(c.grid, c.circles, kind, body,
                                       torch.from_numpy(g).to(DEV), 200)
    gc, gr = G.conform_grad(c.grid, c.circles, 200, g.reshape(2, -1))
    scale = np.abs(gc).max()
    np.testing.assert_allclose(np.array(dcen), gc, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(np.array(drad), gr, rtol=0, atol=1e-12 * np.abs(gr).max())


@pytest.mark.parametrize("c", [SMALL, SMALL_GAP], ids=["five96", "five130_gap0.1"])
def test_copfi_gradient_matches_complex_step(mfp, c):
    say(f"[adjoint full] {c.name}")
    gc, gd = G.complex_step_gradient(c.grid, c.circles, c.flow, c.pair, c.nsweeps)
    # centres from the gap ratio so that torch carries the chain rule to delta
    delta = torch.tensor(c.delta, dtype=torch.float64, requires_grad=True)
    base = torch.tensor([[x, y] for (x, y, _) in c.circles], dtype=torch.float64,
                        requires_grad=True)
    shift = torch.zeros(5, 2, dtype=torch.float64)
    shift[3, 1], shift[4, 1] = -1.0, 1.0
    centres = base + shift * (delta - c.delta)
    radii = [r for (_, _, r) in c.circles]
    J = mfp.copfi(centres, radii, c.grid, c.flow, c.pair, c.nsweeps, "fp64", 1e-13, DEV)
    J.backward()
    g = base.grad.numpy()
    scale = np.abs(gc).max()
    np.testing.assert_allclose(g, gc, rtol=0, atol=1e-7 * scale)
    assert float(delta.grad) == pytest.approx(gd, rel=1e-7)


def test_fp32_refined_adjoint(mfp):
    c = SMALL
    gc, _ = G.complex_step_gradient(c.grid, c.circles, c.flow, c.pair, c.nsweeps,
                                    delta_pair=False)
    centres = torch.tensor([[x, y] for (x, y, _) in c.circles], dtype=torch.float64,
                           requires_grad=True)
    J = mfp.copfi(centres, [r for *_, r in c.circles], c.grid, c.flow, c.pair, c.nsweeps,
                  "fp32_ir", 1e-13, DEV)
    J.backward()
    np.testing.assert_allclose(centres.grad.numpy(), gc, rtol=0,
                               atol=1e-7 * np.abs(gc).max())


def read_gradient_golden():
    """tests/golden/five_cyl_2048x1024_gradient.txt (oracle discrete adjoint, written
    by make_five_cyl_2048_gradient.py): ({key: values}, grad (5, 2))."""
    hdr, rows = {}, []
    with open(os.path.join(HERE, "golden", "five_cyl_2048x1024_gradient.txt")) as f:
        for line in f:
            if line.startswith("#"):
                parts = line[1:].split()
                if parts and parts[0] in ("psi_b", "copfi", "dcopfi_ddelta"):
                    hdr[parts[0]] = np.array([float(v) for v in parts[1:]])
                continue
            b, gx, gy = line.split()
            rows.append((float(gx), float(gy)))
    return hdr, np.array(rows)


def test_full_size_gradient_matches_oracle_and_fd(mfp):
    """2048x1024, delta = 0.15: all 10 centre derivatives and dJ/d(delta) within
    1e-6 max|grad J| of the oracle's discrete-adjoint gradient of the same workload
    (direct sparse-LU solves, tests/golden); dJ/dy of the axis bodies vanish, the
    pair's y derivatives are opposite, x derivatives of the pair equal; dJ/d(delta)
    equals a central difference (step 1e-5) of GPU correction solves warm-started
    from the base solution with an unchanged node classification."""
    c = W.five_cyl_2048_adjoint()
    say("[adjoint full size] forward")
    delta = torch.tensor(c.delta, dtype=torch.float64, requires_grad=True)
    base = torch.tensor([[x, y] for (x, y, _) in c.circles], dtype=torch.float64,
                        requires_grad=True)
    shift = torch.zeros(5, 2, dtype=torch.float64)
    shift[3, 1], shift[4, 1] = -1.0, 1.0
    centres = base + shift * (delta - c.delta)
    radii = [r for (_, _, r) in c.circles]
    J = mfp.copfi(centres, radii, c.grid, c.flow, c.pair, c.nsweeps, "fp64", 1e-13, DEV)
    say("[adjoint full size] backward")
    J.backward()
    g = base.grad.numpy()
    scale = np.abs(g).max()
    assert np.abs(g[:3, 1]).max() <= 1e-9 * scale
    assert g[3, 1] == pytest.approx(-g[4, 1], rel=1e-8)
    assert g[3, 0] == pytest.approx(g[4, 0], rel=1e-6, abs=1e-9 * scale)
    gd = float(delta.grad)
    assert gd == pytest.approx(g[4, 1] - g[3, 1], rel=1e-12)
    hdr, gref = read_gradient_golden()
    bar = 1e-6 * np.abs(gref).max()
    say(f"  vs oracle: centres max {np.abs(g - gref).max():.3e}, delta "
        f"{abs(gd - hdr['dcopfi_ddelta'][0]):.3e} (bar {bar:.2e})")
    np.testing.assert_allclose(g, gref, rtol=0, atol=bar)
    assert abs(gd - hdr["dcopfi_ddelta"][0]) <= bar
    assert float(J.detach()) == pytest.approx(hdr["copfi"][0], abs=1e-10)
    # finite differences of delta with warm-started solves
    say("[adjoint full size] finite differences")
    disp0, kind0, body0 = mfp.mesh_conform(c.grid, c.circles, 200, device=DEV)
    res0 = mfp.psi_solve(c.grid, c.circles, disp0, kind0, body0, c.flow, rtol=1e-13,
                         pair=c.pair)
    h = 1e-5
    vals = []
    for s in (1.0, -1.0):
        cc = [list(x) for x in c.circles]
        cc[3][1] -= s * h
        cc[4][1] += s * h
        cc = [tuple(x) for x in cc]
        disp, kind, body = mfp.mesh_conform(c.grid, cc, 200, device=DEV)
        assert torch.equal(kind, kind0) and torch.equal(body, body0)
        r = mfp.psi_solve(c.grid, cc, disp, kind, body, c.flow, rtol=1e-10, pair=c.pair,
                          psi0=res0.psi, rtol_from_start=True)
        vals.append(r.copfi)
    fd = (vals[0] - vals[1]) / (2 * h)
    assert fd == pytest.approx(gd, rel=1e-6)
