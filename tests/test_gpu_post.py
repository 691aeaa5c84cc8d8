"""GPU parity of the sweep post-processing kernels against the oracle.

mfp_contour (marching squares on the conformed mesh) on the same nodal field as the
oracle's contour: the same segments in the same order, end points within 1e-12
(the crossing interpolations may round differently, e.g. by fused multiply-adds).
Fields: psi of a five-cylinder solve at the transverse bodies' values (their
stagnation streamlines), phi (NaN inside the bodies), a linear field on a conformed
mesh (its level set is an exact straight line), and the benchmark workload's
stagnation streamlines at full size (1024x512).
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import DEV, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mfp():
    need_gpu()
    import paper_2512_12232_amd as m
    m.load()
    return m


def _oracle_mesh(c, disp, kind, body):
    n = c.grid.nodes
    shape = (c.grid.ny + 1, c.grid.nx + 1)
    d = disp.cpu().numpy().reshape(2, *shape)
    return O.Mesh(c.grid, c.circles, kind.cpu().numpy().reshape(shape),
                  body.cpu().numpy().reshape(shape), d)


def _check(mfp, c, disp, kind, body, field, level):
    seg = mfp.contour(c.grid, disp, body, field, level).cpu().numpy()
    ref = O.contour(_oracle_mesh(c, disp, kind, body), field.cpu().numpy(), level)
    assert seg.shape == ref.shape, (seg.shape, ref.shape)
    if len(ref):
        np.testing.assert_allclose(seg, ref, rtol=0, atol=1e-12)
    return seg


def test_stagnation_streamlines_and_equipotentials(mfp):
    c = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    r = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-13, pair=c.pair)
    for b in (3, 4):
        seg = _check(mfp, c, disp, kind, body, r.psi, r.psi_b[b])
        say(f"[contour] psi = psi_{b + 1}: {len(seg)} segments")
        assert len(seg) > 50
    cp = W.potential_flow(c)
    p = mfp.phi_solve(cp.grid, cp.circles, disp, kind, body, cp.flow, rtol=1e-13)
    assert torch.isnan(p.phi).any()
    for level in (-4.0, -0.5, 0.0, 0.5, 3.0):
        _check(mfp, c, disp, kind, body, p.phi, level)


def test_linear_field_is_an_exact_line(mfp):
    c = W.five_cylinders(130, 67, 0.4, extent=(-6.5, 6.5, -3.35, 3.35))
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    mesh = _oracle_mesh(c, disp, kind, body)
    X, Y = mesh.coords()
    f = torch.tensor((0.3 + 0.7 * X - 1.3 * Y).ravel(), device=DEV)
    seg = _check(mfp, c, disp, kind, body, f, 0.1)
    for k in (0, 2):
        np.testing.assert_allclose(0.3 + 0.7 * seg[:, k] - 1.3 * seg[:, k + 1], 0.1,
                                   rtol=0, atol=1e-12)


def test_cap_keeps_the_first_segments(mfp):
    c = W.five_cylinders(96, 48, 0.25, extent=(-6, 6, -3, 3))
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    r = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-12, pair=c.pair)
    full = mfp.contour(c.grid, disp, body, r.psi, r.psi_b[4])
    part = mfp.contour(c.grid, disp, body, r.psi, r.psi_b[4], cap=5)
    assert part.shape == (5, 4) and torch.equal(part, full[:5])


def test_bench_workload_stagnation_streamlines_full_size(mfp):
    c = W.five_cyl_1024()
    disp, kind, body = mfp.mesh_conform(c.grid, c.circles, c.nsweeps, device=DEV)
    r = mfp.psi_solve(c.grid, c.circles, disp, kind, body, c.flow, rtol=1e-12, pair=c.pair)
    for b in (3, 4):
        seg = _check(mfp, c, disp, kind, body, r.psi, r.psi_b[b])
        length = np.hypot(seg[:, 2] - seg[:, 0], seg[:, 3] - seg[:, 1]).sum()
        say(f"[contour] 1024x512 psi = psi_{b + 1}: {len(seg)} segments, length {length:.3f}")
        # the streamline crosses the 40-wide channel and wraps part of the body
        assert 40.0 < length < 45.0
